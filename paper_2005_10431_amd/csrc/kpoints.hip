// Bloch-periodic k-points (Sec. 2.1: Bloch-periodic boundary conditions on
// the orbitals along extended directions, Brillouin-zone integration over
// k-points).
//
// Representation: a complex orbital z = u + i v on the home cell is stored as
// one real column [u ; v] of 2 N_d values.  The complex-linear Hermitian H_k
// acts on such columns as the real symmetric operator [[Re H, -Im H],
// [Im H, Re H]]; a block whose span is closed under z -> i z (the columns
// come in pairs [u; v], [-v; u]) is filtered and Rayleigh-Ritz-rotated by the
// real machinery of the Gamma point with every Bloch eigenvalue appearing
// twice.
//
// H_k z = -1/2 Lap_h^k z + V_eff z + sum_I sum_lm gamma_Il chi~_Ilm <chi~_Ilm, z>,
//   Lap_h^k: the stencil with exp(+-i k_d L_d) on neighbours past the faces;
//   chi~_Ilm(x) = sum_s chi_lm(x + sL - R_I) exp(-i k . sL), over the images s.
#include "internal.hpp"

#include <algorithm>
#include <array>

namespace sg {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kTile = 256;   // points per correction-pass workgroup (one per thread)

struct BlochGeom {
    int nx, ny, nz, no;
    double cx[kMaxHalfOrder + 1], cy[kMaxHalfOrder + 1], cz[kMaxHalfOrder + 1], c0;
    double cph[3], sph[3];   // cos, sin of k_d L_d
    double k[3], L[3], h[3];
    double rc2inv, N0, N1, rcut;
};

BlochGeom bloch_geom(sparc_gpu_ctx c, const double* k) {
    BlochGeom g{};
    g.nx = c->nx;
    g.ny = c->ny;
    g.nz = c->nz;
    g.no = c->n_o;
    for (int q = 0; q <= kMaxHalfOrder; ++q) {
        g.cx[q] = c->cf64.cx[q];
        g.cy[q] = c->cf64.cy[q];
        g.cz[q] = c->cf64.cz[q];
    }
    g.c0 = c->cf64.c0;
    const double L[3] = {c->Lx, c->Ly, c->Lz}, h[3] = {c->hx, c->hy, c->hz};
    for (int d = 0; d < 3; ++d) {
        g.k[d] = k[d];
        g.L[d] = L[d];
        g.h[d] = h[d];
        g.cph[d] = std::cos(k[d] * L[d]);
        g.sph[d] = std::sin(k[d] * L[d]);
    }
    const double rc = c->nl_lmax >= 1 ? c->rc_nl : 1.0;
    g.rc2inv = 1.0 / (rc * rc);
    g.N0 = std::pow(2.0 / (kPi * rc * rc), 0.75);
    g.N1 = (2.0 / rc) * g.N0;
    g.rcut = c->rcut_nl;
    return g;
}

// Scaled Chebyshev recurrence coefficients of step `step` (the same
// recurrence as the Gamma filter): out = alpha (H y - c y) + beta y_prev.
__device__ inline void bloch_coefs(const double* params, int mode, int step, double& alpha, double& cs, double& beta) {
    alpha = 1.0;
    cs = 0.0;
    beta = 0.0;
    if (mode == 0) return;
    const double A = params[0], B = params[1], A0 = params[2];
    const double e = 0.5 * (B - A), c = 0.5 * (B + A);
    const double s1 = e / (A0 - c);
    cs = c;
    if (mode == 1) {
        alpha = s1 / e;
        return;
    }
    const double tau = 2.0 / s1;
    double sp = s1, s = s1;
    for (int k = 2; k <= step; ++k) {
        sp = s;
        s = 1.0 / (tau - s);
    }
    alpha = 2.0 * s / e;
    beta = -sp * s;
}

__device__ inline int floor_div(int i, int n) { return i >= 0 ? i / n : -((-i + n - 1) / n); }

// Projections of NB columns on the complex projectors of one atom:
// proj[(a ncol + col) 8 + r], r < 4: Re, r >= 4: Im of gamma_l dV <chi~_l, z>,
// accumulated over the atom's (point, image) pairs inside rcut.  The pairs
// are those of the Gamma projector tables (flat index and offset in the
// atom's bounding box); the Gaussian, the displacements and the Bloch phase
// exp(i k_d s_d L_d) of the image shift s_d are separable per axis and are
// tabulated in LDS for the box, so a pair costs table reads and the gather.
// U pairs per thread are in flight at once.
template <typename T, int NB, int U>
__global__ __launch_bounds__(256) void k_bloch_proj(const T* __restrict__ X, long ldx, long nd, int ncol,
                                                   const long* __restrict__ ip_off, const int* __restrict__ ip_idx,
                                                   const uint32_t* __restrict__ ip_box,
                                                   const int* __restrict__ box_lo, int ext,
                                                   const double* __restrict__ pos, const double* __restrict__ gamma4,
                                                   const int* __restrict__ atom_order, int n_atoms, BlochGeom g,
                                                   double dV, double* __restrict__ proj) {
    // ex ey ez | dx dy dz | cos_x cos_y cos_z | sin_x sin_y sin_z, ext each
    extern __shared__ double ptab[];
    // Block b runs on XCD b % 8; each XCD takes a contiguous range of the
    // atoms in space-filling order for one column chunk at a time, so the
    // overlapping supports of neighbouring atoms hit in that XCD's L2.
    const int bid = blockIdx.x;
    const int xcd = bid % 8, slot = bid / 8;
    const int per = (n_atoms + 7) / 8;
    const int rank = xcd * per + slot % per;
    const int chunk = slot / per;
    if (rank >= n_atoms || chunk * NB >= ncol) return;
    const int a = atom_order[rank];
    const int col0 = chunk * NB;
    const int nt = blockDim.x;
    for (int q = threadIdx.x; q < 3 * ext; q += nt) {
        const int d = q / ext, i = q - d * ext;
        const int gi = box_lo[3 * a + d] + i;
        const double dv = gi * g.h[d] - pos[3 * a + d];
        ptab[q] = exp(-dv * dv * g.rc2inv);
        ptab[3 * ext + q] = dv;
        const int sd = floor_div(gi, d == 0 ? g.nx : (d == 1 ? g.ny : g.nz));
        double sn, cs;
        sincos(g.k[d] * sd * g.L[d], &sn, &cs);
        ptab[6 * ext + q] = cs;
        ptab[9 * ext + q] = sn;
    }
    __syncthreads();
    const double* ex = ptab;
    const double* ey = ptab + ext;
    const double* ez = ptab + 2 * ext;
    const double* dxt = ptab + 3 * ext;
    const double* dyt = ptab + 4 * ext;
    const double* dzt = ptab + 5 * ext;
    const double* cxt = ptab + 6 * ext;
    const double* cyt = ptab + 7 * ext;
    const double* czt = ptab + 8 * ext;
    const double* sxt = ptab + 9 * ext;
    const double* syt = ptab + 10 * ext;
    const double* szt = ptab + 11 * ext;
    const int nb = min(NB, ncol - col0);
    double acc[NB * 8];
#pragma unroll
    for (int q = 0; q < NB * 8; ++q) acc[q] = 0.0;
    const long s0 = ip_off[a], s1 = ip_off[a + 1];
    for (long s = s0 + threadIdx.x; s < s1; s += (long)U * nt) {
        long idx[U];
        uint32_t bb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long su = s + (long)u * nt;
            const bool ok = su < s1;
            idx[u] = ok ? ip_idx[su] : 0;
            bb[u] = ok ? ip_box[su] : 0xFFFFFFFFu;
        }
        double xu[U][NB], xv[U][NB];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                const bool ok = bb[u] != 0xFFFFFFFFu && c < nb;
                const long o = idx[u] + (long)(col0 + c) * ldx;
                xu[u][c] = ok ? (double)X[o] : 0.0;
                xv[u][c] = ok ? (double)X[nd + o] : 0.0;
            }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (bb[u] == 0xFFFFFFFFu) break;
            const uint32_t b = bb[u];
            const int bx = b & 0xFF, by = (b >> 8) & 0xFF, bz = (b >> 16) & 0xFF;
            const double e = ex[bx] * ey[by] * ez[bz];
            const double chi[4] = {g.N0 * e, g.N1 * dxt[bx] * e, g.N1 * dyt[by] * e, g.N1 * dzt[bz] * e};
            // exp(i (theta_x + theta_y + theta_z)) as a product of the axis factors
            const double cxy = cxt[bx] * cyt[by] - sxt[bx] * syt[by];
            const double sxy = sxt[bx] * cyt[by] + cxt[bx] * syt[by];
            const double cs = cxy * czt[bz] - sxy * szt[bz];
            const double sn = sxy * czt[bz] + cxy * szt[bz];
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                if (c < nb) {
                    // conj(chi~) z = chi exp(+i theta) (u + i v)
                    const double zr = cs * xu[u][c] - sn * xv[u][c], zi = sn * xu[u][c] + cs * xv[u][c];
#pragma unroll
                    for (int l = 0; l < 4; ++l) {
                        acc[8 * c + l] += chi[l] * zr;
                        acc[8 * c + 4 + l] += chi[l] * zi;
                    }
                }
            }
        }
    }
    __shared__ double lds[4][NB * 8];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NB * 8; ++q) {
        double t = acc[q];
        for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
        if (lane == 0) lds[w][q] = t;
    }
    __syncthreads();
    const int q = threadIdx.x;
    if (q < NB * 8) {
        const int c = q / 8, r = q % 8;
        if (col0 + c < ncol) {
            const double sum = ((lds[0][q] + lds[1][q]) + lds[2][q]) + lds[3][q];
            proj[((long)a * ncol + col0 + c) * 8 + r] = dV * gamma4[4 * a + (r & 3)] * sum;
        }
    }
}

// out = alpha (H_k y - c y) + beta prev for every point of every column
// (mode 0: out = H_k y).  out may alias prev (each element is read before it
// is written, by the same thread); y must not alias either.
template <typename T>
__global__ __launch_bounds__(256) void k_bloch_apply(const T* __restrict__ Y, T* out, const T* prev, long ldx, long nd,
                                                    const double* __restrict__ veff, BlochGeom g,
                                                    const double* __restrict__ proj, int ncol,
                                                    const int* __restrict__ off, const uint32_t* __restrict__ ent,
                                                    const double* __restrict__ pos,
                                                    const double* __restrict__ params, int mode, int step) {
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int col = blockIdx.y;
    if (p >= nd) return;
    const int nx = g.nx, ny = g.ny;
    const long nxy = (long)nx * ny;
    const int ix = (int)(p % nx), iy = (int)((p / nx) % ny), iz = (int)(p / nxy);
    const T* yu = Y + (long)col * ldx;
    const T* yv = yu + nd;
    const double u0 = (double)yu[p], v0 = (double)yv[p];
    double lu = g.c0 * u0, lv = g.c0 * v0;
    // one axis: neighbours at +-q with stride `st`; past a face the value is
    // the image's, times exp(+-i k L) on that axis
    auto axis = [&](int i, int n, long st, long span, const double* cf, double cph, double sph) {
        for (int q = 1; q <= g.no; ++q) {
            const double w = cf[q];
            if (i + q < n) {
                lu += w * (double)yu[p + q * st];
                lv += w * (double)yv[p + q * st];
            } else {
                const long pp = p + q * st - span;
                const double a = (double)yu[pp], b = (double)yv[pp];
                lu += w * (a * cph - b * sph);
                lv += w * (a * sph + b * cph);
            }
            if (i - q >= 0) {
                lu += w * (double)yu[p - q * st];
                lv += w * (double)yv[p - q * st];
            } else {
                const long pp = p - q * st + span;
                const double a = (double)yu[pp], b = (double)yv[pp];
                lu += w * (a * cph + b * sph);
                lv += w * (-a * sph + b * cph);
            }
        }
    };
    axis(ix, nx, 1, nx, g.cx, g.cph[0], g.sph[0]);
    axis(iy, ny, nx, nxy, g.cy, g.cph[1], g.sph[1]);
    axis(iz, g.nz, nxy, nd, g.cz, g.cph[2], g.sph[2]);
    double hu = lu + veff[p] * u0, hv = lv + veff[p] * v0;
    if (proj) {
        for (int e = off[p]; e < off[p + 1]; ++e) {
            const uint32_t w = ent[e];
            const int a = (int)(w & 0xFFFFFu);
            const int sx = (int)((w >> 20) & 15u) - 8, sy = (int)((w >> 24) & 15u) - 8, sz = (int)(w >> 28) - 8;
            const double dx = (ix + sx * nx) * g.h[0] - pos[3 * a];
            const double dy = (iy + sy * ny) * g.h[1] - pos[3 * a + 1];
            const double dz = (iz + sz * g.nz) * g.h[2] - pos[3 * a + 2];
            const double ex = exp(-(dx * dx + dy * dy + dz * dz) * g.rc2inv);
            const double c0 = g.N0 * ex, c1 = g.N1 * dx * ex, c2 = g.N1 * dy * ex, c3 = g.N1 * dz * ex;
            const double* C = proj + ((long)a * ncol + col) * 8;
            const double cre = c0 * C[0] + c1 * C[1] + c2 * C[2] + c3 * C[3];
            const double cim = c0 * C[4] + c1 * C[5] + c2 * C[6] + c3 * C[7];
            double sn, cs;
            sincos(g.k[0] * sx * g.L[0] + g.k[1] * sy * g.L[1] + g.k[2] * sz * g.L[2], &sn, &cs);
            // chi~ C = chi exp(-i theta) (cre + i cim)
            hu += cre * cs + cim * sn;
            hv += cim * cs - cre * sn;
        }
    }
    double alpha, cs, beta;
    bloch_coefs(params, mode, step, alpha, cs, beta);
    double ou = alpha * (hu - cs * u0), ov = alpha * (hv - cs * v0);
    const long o = (long)col * ldx + p;
    if (mode == 2) {
        ou += beta * (double)prev[o];
        ov += beta * (double)prev[o + nd];
    }
    out[o] = (T)ou;
    out[o + nd] = (T)ov;
}

// Projector values and Bloch phase of every (point, atom, image) entry at
// one k: et[6 e] = chi_s, chi_px, chi_py, chi_pz, cos(k . sL), sin(k . sL).
__global__ void k_bloch_entry_table(const int* __restrict__ off, const uint32_t* __restrict__ ent, long nd,
                                    const double* __restrict__ pos, BlochGeom g, double* __restrict__ et) {
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nd) return;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const long nxy = (long)nx * ny;
    const int ix = (int)(p % nx), iy = (int)((p / nx) % ny), iz = (int)(p / nxy);
    for (int e = off[p]; e < off[p + 1]; ++e) {
        const uint32_t w = ent[e];
        const int a = (int)(w & 0xFFFFFu);
        const int sx = (int)((w >> 20) & 15u) - 8, sy = (int)((w >> 24) & 15u) - 8, sz = (int)(w >> 28) - 8;
        const double dx = (ix + sx * nx) * g.h[0] - pos[3 * a];
        const double dy = (iy + sy * ny) * g.h[1] - pos[3 * a + 1];
        const double dz = (iz + sz * nz) * g.h[2] - pos[3 * a + 2];
        const double ex = exp(-(dx * dx + dy * dy + dz * dz) * g.rc2inv);
        double sn, cs;
        sincos(g.k[0] * sx * g.L[0] + g.k[1] * sy * g.L[1] + g.k[2] * sz * g.L[2], &sn, &cs);
        double* o = et + 6L * e;
        o[0] = g.N0 * ex;
        o[1] = g.N1 * dx * ex;
        o[2] = g.N1 * dy * ex;
        o[3] = g.N1 * dz * ex;
        o[4] = cs;
        o[5] = sn;
    }
}

// Bloch terms on top of the Gamma local sweep (which applied the periodic
// real stencil and V_eff to u and v separately and the filter recurrence):
// out += alpha (boundary phase corrections + phased nonlocal term), only at
// points within the stencil's reach of a face or inside a projector support.
// Each thread serves NC columns, so the projector values and phases of a
// point's entries are evaluated once for all of them.
template <typename T, int NC>
__global__ __launch_bounds__(256) void k_bloch_fix(const T* __restrict__ Y, T* __restrict__ out, long ldx, long nd,
                                                  BlochGeom g, const double* __restrict__ proj, int ncol,
                                                  const int* __restrict__ off, const uint32_t* __restrict__ ent,
                                                  const uint16_t* __restrict__ slot,
                                                  const int* __restrict__ tile_off,
                                                  const int* __restrict__ tile_atoms,
                                                  const double* __restrict__ et,
                                                  const double* __restrict__ params, int mode, int step) {
    // the tile's projection coefficients for its NC columns, staged in LDS:
    // cl[(slot NC + c) 8 + r]
    extern __shared__ double cl[];
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int col0 = blockIdx.y * NC;
    const int nc = min(NC, ncol - col0);
    if (proj) {
        const int t0 = tile_off[blockIdx.x], na = tile_off[blockIdx.x + 1] - t0;
        for (int q = threadIdx.x; q < na * NC * 8; q += blockDim.x) {
            const int sl = q / (NC * 8), c = (q / 8) % NC, r = q % 8;
            cl[q] = c < nc ? proj[((long)tile_atoms[t0 + sl] * ncol + col0 + c) * 8 + r] : 0.0;
        }
        __syncthreads();
    }
    if (p >= nd) return;
    const int nx = g.nx, ny = g.ny, nz = g.nz, no = g.no;
    const long nxy = (long)nx * ny;
    const int ix = (int)(p % nx), iy = (int)((p / nx) % ny), iz = (int)(p / nxy);
    const bool edge = ix < no || ix >= nx - no || iy < no || iy >= ny - no || iz < no || iz >= nz - no;
    const bool has_nl = proj && off[p + 1] > off[p];
    if (!edge && !has_nl) return;
    double cu[NC], cv[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) cu[c] = cv[c] = 0.0;
    if (edge) {
        // the sweep used y(wrapped); the Bloch value is y(wrapped) exp(+-i k L)
        auto axis = [&](int i, int n, long st, long span, const double* cf, double cph, double sph) {
            for (int q = 1; q <= no; ++q) {
                const double w = cf[q];
                if (i + q >= n) {
                    const long pp = p + q * st - span;
#pragma unroll
                    for (int c = 0; c < NC; ++c)
                        if (c < nc) {
                            const T* yu = Y + (long)(col0 + c) * ldx;
                            const double a = (double)yu[pp], b = (double)yu[nd + pp];
                            cu[c] += w * (a * (cph - 1.0) - b * sph);
                            cv[c] += w * (a * sph + b * (cph - 1.0));
                        }
                }
                if (i - q < 0) {
                    const long pp = p - q * st + span;
#pragma unroll
                    for (int c = 0; c < NC; ++c)
                        if (c < nc) {
                            const T* yu = Y + (long)(col0 + c) * ldx;
                            const double a = (double)yu[pp], b = (double)yu[nd + pp];
                            cu[c] += w * (a * (cph - 1.0) + b * sph);
                            cv[c] += w * (-a * sph + b * (cph - 1.0));
                        }
                }
            }
        };
        axis(ix, nx, 1, nx, g.cx, g.cph[0], g.sph[0]);
        axis(iy, ny, nx, nxy, g.cy, g.cph[1], g.sph[1]);
        axis(iz, nz, nxy, nd, g.cz, g.cph[2], g.sph[2]);
    }
    if (has_nl) {
        for (int e = off[p]; e < off[p + 1]; ++e) {
            const double* te = et + 6L * e;
            const double c0 = te[0], c1 = te[1], c2 = te[2], c3 = te[3], cs = te[4], sn = te[5];
            const double* Cb = cl + (long)slot[e] * NC * 8;
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (c < nc) {
                    const double* C = Cb + 8 * c;
                    const double cre = c0 * C[0] + c1 * C[1] + c2 * C[2] + c3 * C[3];
                    const double cim = c0 * C[4] + c1 * C[5] + c2 * C[6] + c3 * C[7];
                    cu[c] += cre * cs + cim * sn;
                    cv[c] += cim * cs - cre * sn;
                }
        }
    }
    double alpha, csh, beta;
    bloch_coefs(params, mode, step, alpha, csh, beta);
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (c < nc) {
            const long o = (long)(col0 + c) * ldx + p;
            out[o] = (T)((double)out[o] + alpha * cu[c]);
            out[o + nd] = (T)((double)out[o + nd] + alpha * cv[c]);
        }
}

// columns per thread of the correction pass: 72 VGPRs, 7 waves per SIMD (8 and 2 were slower)
constexpr int kFixNC = 4;

template <typename T>
__global__ void k_copy_block_k(const T* __restrict__ src, T* __restrict__ dst, long rows, int ncol, long ld) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i < rows && j < ncol) dst[i + (long)j * ld] = src[i + (long)j * ld];
}

constexpr int kProjNB = 4;

}  // namespace

// Point-major (atom, image) entries of the projector supports: for grid
// point p, entries off[p] .. off[p+1] of ent, each packing the atom (20 bits)
// and its image offset s + 8 per axis (4 bits each).
sparc_status ensure_kp_tables(sparc_gpu_ctx c) {
    if (c->kp_off || c->nl_lmax < 1) return SPARC_OK;
    const int n = c->n_atoms;
    if (n >= (1 << 20)) return set_err(c, SPARC_ERR_ARG, "k-points: too many atoms for the entry tables");
    const double h[3] = {c->hx, c->hy, c->hz};
    const int N[3] = {c->nx, c->ny, c->nz};
    const double rc = c->rcut_nl;
    std::vector<std::pair<long, uint32_t>> list;
    for (int a = 0; a < n; ++a) {
        int lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
            lo[d] = (int)std::ceil((c->pos[3 * a + d] - rc) / h[d]);
            hi[d] = (int)std::floor((c->pos[3 * a + d] + rc) / h[d]);
        }
        for (int k = lo[2]; k <= hi[2]; ++k)
            for (int j = lo[1]; j <= hi[1]; ++j)
                for (int i = lo[0]; i <= hi[0]; ++i) {
                    const double dx = i * h[0] - c->pos[3 * a], dy = j * h[1] - c->pos[3 * a + 1];
                    const double dz = k * h[2] - c->pos[3 * a + 2];
                    if (dx * dx + dy * dy + dz * dz > rc * rc) continue;
                    const int ii[3] = {i, j, k};
                    int s[3], w[3];
                    for (int d = 0; d < 3; ++d) {
                        s[d] = ii[d] >= 0 ? ii[d] / N[d] : -((-ii[d] + N[d] - 1) / N[d]);
                        w[d] = ii[d] - s[d] * N[d];
                        if (s[d] < -8 || s[d] > 7)
                            return set_err(c, SPARC_ERR_ARG, "k-points: projector support spans too many images");
                    }
                    const long flat = w[0] + (long)N[0] * (w[1] + (long)N[1] * w[2]);
                    const uint32_t code = (uint32_t)a | ((uint32_t)(s[0] + 8) << 20) | ((uint32_t)(s[1] + 8) << 24) |
                                          ((uint32_t)(s[2] + 8) << 28);
                    list.push_back({flat, code});
                }
    }
    if (list.size() >= (size_t)1 << 31) return set_err(c, SPARC_ERR_ARG, "k-points: too many projector entries");
    std::vector<int> off(c->nd + 1, 0);
    for (auto& e : list) off[e.first + 1]++;
    for (long p = 0; p < c->nd; ++p) off[p + 1] += off[p];
    std::vector<uint32_t> ent(list.size());
    std::vector<int> fill(off.begin(), off.end() - 1);
    for (auto& e : list) ent[fill[e.first]++] = e.second;
    // tiles of kTile consecutive points: the distinct atoms of their entries,
    // and for each entry the atom's position in its tile's list
    const long ntile = (c->nd + kTile - 1) / kTile;
    std::vector<int> toff(ntile + 1, 0), tatoms;
    std::vector<uint16_t> slot(ent.size());
    int tmax = 0;
    for (long t = 0; t < ntile; ++t) {
        const long p0 = t * kTile, p1 = std::min<long>(c->nd, p0 + kTile);
        std::vector<int> atoms_t;
        for (int e = off[p0]; e < off[p1]; ++e) atoms_t.push_back((int)(ent[e] & 0xFFFFFu));
        std::sort(atoms_t.begin(), atoms_t.end());
        atoms_t.erase(std::unique(atoms_t.begin(), atoms_t.end()), atoms_t.end());
        if (atoms_t.size() > 65535) return set_err(c, SPARC_ERR_ARG, "k-points: too many atoms in one tile");
        for (int e = off[p0]; e < off[p1]; ++e)
            slot[e] = (uint16_t)(std::lower_bound(atoms_t.begin(), atoms_t.end(), (int)(ent[e] & 0xFFFFFu)) -
                                 atoms_t.begin());
        tatoms.insert(tatoms.end(), atoms_t.begin(), atoms_t.end());
        toff[t + 1] = (int)tatoms.size();
        tmax = std::max(tmax, (int)atoms_t.size());
    }
    SG_HIP(c, hipMalloc((void**)&c->kp_off, off.size() * sizeof(int)));
    SG_HIP(c, hipMalloc((void**)&c->kp_ent, std::max<size_t>(1, ent.size()) * sizeof(uint32_t)));
    SG_HIP(c, hipMalloc((void**)&c->kp_slot, std::max<size_t>(1, slot.size()) * sizeof(uint16_t)));
    SG_HIP(c, hipMalloc((void**)&c->kp_tile_off, toff.size() * sizeof(int)));
    SG_HIP(c, hipMalloc((void**)&c->kp_tile_atoms, std::max<size_t>(1, tatoms.size()) * sizeof(int)));
    SG_HIP(c, hipMemcpy(c->kp_off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice));
    SG_HIP(c, hipMemcpy(c->kp_tile_off, toff.data(), toff.size() * sizeof(int), hipMemcpyHostToDevice));
    if (!ent.empty()) {
        SG_HIP(c, hipMemcpy(c->kp_ent, ent.data(), ent.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
        SG_HIP(c, hipMemcpy(c->kp_slot, slot.data(), slot.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
        SG_HIP(c, hipMemcpy(c->kp_tile_atoms, tatoms.data(), tatoms.size() * sizeof(int), hipMemcpyHostToDevice));
    }
    c->kp_tile_max = tmax;
    c->kp_n_ent = (long)ent.size();
    return SPARC_OK;
}

// Signed nonlocal bounds at k: sum over atoms and lm of min/max(gamma, 0)
// dV ||chi~_lm||^2 (the k-dependent projector norms), cached per k.
sparc_status kp_nl_bounds(sparc_gpu_ctx c, const double* k, double* nl_lo, double* nl_hi) {
    *nl_lo = *nl_hi = 0.0;
    if (c->nl_lmax < 1) return SPARC_OK;
    for (auto& e : c->kp_bound_cache)
        if (e[0] == k[0] && e[1] == k[1] && e[2] == k[2]) {
            *nl_lo = e[3];
            *nl_hi = e[4];
            return SPARC_OK;
        }
    const double h[3] = {c->hx, c->hy, c->hz}, L[3] = {c->Lx, c->Ly, c->Lz};
    const int N[3] = {c->nx, c->ny, c->nz};
    const double rc = c->rc_nl, rcut = c->rcut_nl;
    const double N0 = std::pow(2.0 / (kPi * rc * rc), 0.75), N1 = (2.0 / rc) * N0;
    double lo = 0.0, hi = 0.0;
    for (int a = 0; a < c->n_atoms; ++a) {
        std::vector<std::pair<long, std::array<double, 8>>> pts;
        int l0[3], h0[3];
        for (int d = 0; d < 3; ++d) {
            l0[d] = (int)std::ceil((c->pos[3 * a + d] - rcut) / h[d]);
            h0[d] = (int)std::floor((c->pos[3 * a + d] + rcut) / h[d]);
        }
        for (int kk = l0[2]; kk <= h0[2]; ++kk)
            for (int j = l0[1]; j <= h0[1]; ++j)
                for (int i = l0[0]; i <= h0[0]; ++i) {
                    const int ii[3] = {i, j, kk};
                    double dd[3], r2 = 0.0;
                    for (int d = 0; d < 3; ++d) {
                        dd[d] = ii[d] * h[d] - c->pos[3 * a + d];
                        r2 += dd[d] * dd[d];
                    }
                    if (r2 > rcut * rcut) continue;
                    int s[3], w[3];
                    double th = 0.0;
                    for (int d = 0; d < 3; ++d) {
                        s[d] = ii[d] >= 0 ? ii[d] / N[d] : -((-ii[d] + N[d] - 1) / N[d]);
                        w[d] = ii[d] - s[d] * N[d];
                        th += k[d] * s[d] * L[d];
                    }
                    const double ex = std::exp(-r2 / (rc * rc));
                    const double chi[4] = {N0 * ex, N1 * dd[0] * ex, N1 * dd[1] * ex, N1 * dd[2] * ex};
                    std::array<double, 8> v;
                    for (int l = 0; l < 4; ++l) {
                        v[l] = chi[l] * std::cos(th);
                        v[4 + l] = -chi[l] * std::sin(th);
                    }
                    pts.push_back({w[0] + (long)N[0] * (w[1] + (long)N[1] * w[2]), v});
                }
        std::sort(pts.begin(), pts.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
        double nrm[4] = {0, 0, 0, 0};
        for (size_t b = 0; b < pts.size();) {
            std::array<double, 8> s{};
            size_t e = b;
            for (; e < pts.size() && pts[e].first == pts[b].first; ++e)
                for (int r = 0; r < 8; ++r) s[r] += pts[e].second[r];
            for (int l = 0; l < 4; ++l) nrm[l] += s[l] * s[l] + s[4 + l] * s[4 + l];
            b = e;
        }
        const double g[4] = {c->gamma[2 * a], c->gamma[2 * a + 1], c->gamma[2 * a + 1], c->gamma[2 * a + 1]};
        for (int l = 0; l < 4; ++l) {
            lo += std::min(g[l], 0.0) * c->dV * nrm[l];
            hi += std::max(g[l], 0.0) * c->dV * nrm[l];
        }
    }
    c->kp_bound_cache.push_back({k[0], k[1], k[2], lo, hi});
    *nl_lo = lo;
    *nl_hi = hi;
    return SPARC_OK;
}

static sparc_status ensure_kp_proj(sparc_gpu_ctx c, size_t elems) {
    if (c->kp_proj_elems >= elems) return SPARC_OK;
    if (c->kp_proj) {
        SG_HIP(c, hipStreamSynchronize(c->stream));
        SG_HIP(c, hipFree(c->kp_proj));
        c->kp_proj = nullptr;
        c->kp_proj_elems = 0;
    }
    SG_HIP(c, hipMalloc((void**)&c->kp_proj, elems * sizeof(double)));
    c->kp_proj_elems = elems;
    return SPARC_OK;
}

// One application of H_k (mode 0) or one filter step (modes 1, 2) at the
// context's current k; projections first when the system has projectors.
template <typename T>
static sparc_status bloch_step(sparc_gpu_ctx c, const T* Y, T* out, const T* prev, int ncol, long ldx, int mode,
                               int step) {
    sparc_status st;
    const BlochGeom g = bloch_geom(c, c->kvec);
    const bool nl = c->nl_lmax >= 1;
    double* proj = nullptr;
    if (nl) {
        if ((st = ensure_force_tables(c)) != SPARC_OK) return st;
        if ((st = ensure_kp_tables(c)) != SPARC_OK) return st;
        if ((st = ensure_kp_proj(c, (size_t)c->n_atoms * ncol * 8)) != SPARC_OK) return st;
        proj = c->kp_proj;
        const int slot = prof_begin(c, PK_BLOCH_PROJ);
        const int n = c->n_atoms;
        const int ext = std::max(1, c->nl.box_ext);
        const int per = (n + 7) / 8;
        k_bloch_proj<T, kProjNB, 2><<<dim3(8 * per * div_up(ncol, kProjNB)), 256, 12 * ext * sizeof(double),
                                      c->stream>>>(Y, ldx, c->nd, ncol, c->nl.ip_off, c->nl.ip_idx, c->nl.ip_box,
                                                   c->nl.box_lo, ext, c->force_tab, c->force_tab + 5 * n,
                                                   c->nl.atom_order, n, g, c->dV, proj);
        SG_CHECK_LAUNCH(c);
        prof_end(c, slot);
    }
    const int slot = prof_begin(c, PK_BLOCH);
    // correction pass LDS: the coefficients of a tile's atoms for kFixNC columns
    const size_t lds = nl ? (size_t)c->kp_tile_max * kFixNC * 8 * sizeof(double) : 0;
    if (ldx == 2 * c->nd && lds <= 64 * 1024) {
        // unpadded blocks: the halves u, v are real columns of N_d rows, swept
        // by the Gamma local kernel (recurrence fused); then the Bloch terms
        c->sweep_local_only = 1;
        st = launch_hsweep<T>(c, Y, out, prev, 2 * ncol, c->nd, mode, step);
        c->sweep_local_only = 0;
        if (st != SPARC_OK) return st;
        if (nl && !(c->kp_etab_valid && c->kp_etab_k[0] == c->kvec[0] && c->kp_etab_k[1] == c->kvec[1] &&
                    c->kp_etab_k[2] == c->kvec[2])) {
            if (!c->kp_etab) SG_HIP(c, hipMalloc((void**)&c->kp_etab, 6 * std::max(1L, c->kp_n_ent) * sizeof(double)));
            k_bloch_entry_table<<<div_up(c->nd, 256), 256, 0, c->stream>>>(c->kp_off, c->kp_ent, c->nd, c->force_tab,
                                                                           g, c->kp_etab);
            for (int d = 0; d < 3; ++d) c->kp_etab_k[d] = c->kvec[d];
            c->kp_etab_valid = 1;
        }
        k_bloch_fix<T, kFixNC><<<dim3(div_up(c->nd, kTile), div_up(ncol, kFixNC)), kTile, lds, c->stream>>>(
            Y, out, ldx, c->nd, g, proj, ncol, c->kp_off, c->kp_ent, c->kp_slot, c->kp_tile_off, c->kp_tile_atoms,
            c->kp_etab, c->scal + S_A, mode, step);
    } else {
        k_bloch_apply<T><<<dim3(div_up(c->nd, 256), ncol), 256, 0, c->stream>>>(
            Y, out, prev, ldx, c->nd, c->veff, g, proj, ncol, c->kp_off, c->kp_ent, nl ? c->force_tab : nullptr,
            c->scal + S_A, mode, step);
    }
    SG_CHECK_LAUNCH(c);
    prof_end(c, slot);
    return SPARC_OK;
}

template <typename T>
sparc_status bloch_apply_impl(sparc_gpu_ctx c, const T* X, T* Y, int ncol, long ldx) {
    return bloch_step<T>(c, X, Y, nullptr, ncol, ldx, 0, 0);
}
template sparc_status bloch_apply_impl<double>(sparc_gpu_ctx, const double*, double*, int, long);
template sparc_status bloch_apply_impl<float>(sparc_gpu_ctx, const float*, float*, int, long);

// Filter with bounds in c->scal[S_A..S_A0]: Y_k in X for even k, in W for
// odd k; the result ends in X (the Gamma filter's schedule).
template <typename T>
sparc_status bloch_filter_impl(sparc_gpu_ctx c, T* X, T* W, int ncol, long ldx, int m) {
    sparc_status st;
    if ((st = bloch_step<T>(c, X, W, nullptr, ncol, ldx, 1, 1)) != SPARC_OK) return st;
    for (int k = 2; k <= m; ++k) {
        T* cur = (k % 2 == 0) ? W : X;
        T* dst = (k % 2 == 0) ? X : W;
        if ((st = bloch_step<T>(c, cur, dst, dst, ncol, ldx, 2, k)) != SPARC_OK) return st;
    }
    if (m % 2 == 1) {
        k_copy_block_k<T><<<dim3(div_up(2 * c->nd, 256), ncol), 256, 0, c->stream>>>(W, X, 2 * c->nd, ncol, ldx);
        SG_CHECK_LAUNCH(c);
    }
    return SPARC_OK;
}
template sparc_status bloch_filter_impl<double>(sparc_gpu_ctx, double*, double*, int, long, int);
template sparc_status bloch_filter_impl<float>(sparc_gpu_ctx, float*, float*, int, long, int);

// Spectrum bounds of H_k into S_LO / S_HI (V_eff extrema plus the
// k-dependent nonlocal bounds).
sparc_status bloch_bounds_impl(sparc_gpu_ctx c) {
    double lo, hi;
    sparc_status st = kp_nl_bounds(c, c->kvec, &lo, &hi);
    if (st != SPARC_OK) return st;
    // the Gamma routine with the k-dependent nonlocal terms (its kernels take
    // them as launch arguments)
    const double glo = c->nl.nl_lo, ghi = c->nl.nl_hi;
    c->nl.nl_lo = lo;
    c->nl.nl_hi = hi;
    st = bounds_impl(c);
    c->nl.nl_lo = glo;
    c->nl.nl_hi = ghi;
    return st;
}

}  // namespace sg

using namespace sg;

namespace {

__global__ void k_set_params3(double* dst, double a, double b, double c) {
    dst[0] = a;
    dst[1] = b;
    dst[2] = c;
}

sparc_status check_k_block(sparc_gpu_ctx c, const double* k, int prec, const void* X, int ncol, long ldx,
                           const char* who) {
    if (!k || !std::isfinite(k[0]) || !std::isfinite(k[1]) || !std::isfinite(k[2]))
        return set_err(c, SPARC_ERR_ARG, std::string(who) + ": bad k");
    if (prec != SPARC_FP64 && prec != SPARC_FP32) return set_err(c, SPARC_ERR_ARG, std::string(who) + ": bad precision");
    if (!X) return set_err(c, SPARC_ERR_ARG, std::string(who) + ": null block");
    if (ncol < 1 || ncol > 2 * c->n_states)
        return set_err(c, SPARC_ERR_ARG, std::string(who) + ": ncol outside [1, 2 n_states]");
    if (ldx < 2 * c->nd) return set_err(c, SPARC_ERR_ARG, std::string(who) + ": ldx < 2 N_d");
    return SPARC_OK;
}

bool blocks_overlap(const void* a, const void* b, size_t bytes) {
    const char* pa = (const char*)a;
    const char* pb = (const char*)b;
    return pa < pb + bytes && pb < pa + bytes;
}

void set_k(sparc_gpu_ctx c, const double* k) {
    for (int d = 0; d < 3; ++d) c->kvec[d] = k[d];
}

}  // namespace

extern "C" {

sparc_status sparc_gpu_apply_H_k(sparc_gpu_ctx c, const double* k, sparc_prec prec, const void* d_X, void* d_Y,
                                 int ncol, long ldx) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    sparc_status st = check_k_block(c, k, prec, d_X, ncol, ldx, "apply_H_k");
    if (st != SPARC_OK) return st;
    if (!d_Y) return set_err(c, SPARC_ERR_ARG, "apply_H_k: null output");
    const size_t es = prec == SPARC_FP64 ? 8 : 4;
    if (blocks_overlap(d_X, d_Y, ((size_t)(ncol - 1) * ldx + 2 * c->nd) * es))
        return set_err(c, SPARC_ERR_ARG, "apply_H_k: X and Y overlap");
    set_k(c, k);
    if (prec == SPARC_FP64) return bloch_apply_impl<double>(c, (const double*)d_X, (double*)d_Y, ncol, ldx);
    return bloch_apply_impl<float>(c, (const float*)d_X, (float*)d_Y, ncol, ldx);
}

sparc_status sparc_gpu_chebyshev_filter_k(sparc_gpu_ctx c, const double* k, sparc_prec prec, void* d_X, void* d_work,
                                          int ncol, long ldx, int degree, double a, double b, double a0) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    sparc_status st = check_k_block(c, k, prec, d_X, ncol, ldx, "chebyshev_filter_k");
    if (st != SPARC_OK) return st;
    if (!d_work) return set_err(c, SPARC_ERR_ARG, "chebyshev_filter_k: null work block");
    if (degree < 1 || degree > 10000) return set_err(c, SPARC_ERR_ARG, "chebyshev_filter_k: degree out of range");
    if (!(a0 < a && a < b) || !std::isfinite(a0) || !std::isfinite(b))
        return set_err(c, SPARC_ERR_ARG, "chebyshev_filter_k: need a0 < a < b");
    const size_t es = prec == SPARC_FP64 ? 8 : 4;
    if (blocks_overlap(d_X, d_work, ((size_t)(ncol - 1) * ldx + 2 * c->nd) * es))
        return set_err(c, SPARC_ERR_ARG, "chebyshev_filter_k: X and work overlap");
    set_k(c, k);
    k_set_params3<<<1, 1, 0, c->stream>>>(c->scal + S_A, a, b, a0);
    SG_CHECK_LAUNCH(c);
    if (prec == SPARC_FP64) return bloch_filter_impl<double>(c, (double*)d_X, (double*)d_work, ncol, ldx, degree);
    return bloch_filter_impl<float>(c, (float*)d_X, (float*)d_work, ncol, ldx, degree);
}

sparc_status sparc_gpu_rayleigh_ritz_k(sparc_gpu_ctx c, const double* k, sparc_prec prec, void* d_X, int ncol,
                                       long ldx, double* d_eig) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    sparc_status st = check_k_block(c, k, prec, d_X, ncol, ldx, "rayleigh_ritz_k");
    if (st != SPARC_OK) return st;
    if (!d_eig) return set_err(c, SPARC_ERR_ARG, "rayleigh_ritz_k: null eigenvalue output");
    if (ncol > kEighMaxN) return set_err(c, SPARC_ERR_ARG, "rayleigh_ritz_k: ncol above the eigensolver limit");
    set_k(c, k);
    if (prec == SPARC_FP64) return rayleigh_ritz_k_impl<double>(c, (double*)d_X, ncol, ldx, d_eig, true);
    return rayleigh_ritz_k_impl<float>(c, (float*)d_X, ncol, ldx, d_eig, true);
}

sparc_status sparc_gpu_spectrum_bounds_k(sparc_gpu_ctx c, const double* k, double* lo, double* hi) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    if (!k || !std::isfinite(k[0]) || !std::isfinite(k[1]) || !std::isfinite(k[2]))
        return set_err(c, SPARC_ERR_ARG, "spectrum_bounds_k: bad k");
    set_k(c, k);
    sparc_status st = bloch_bounds_impl(c);
    if (st != SPARC_OK) return st;
    double h2[2];
    SG_HIP(c, hipMemcpyAsync(h2, c->scal + S_LO, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    SG_HIP(c, hipStreamSynchronize(c->stream));
    if (lo) *lo = h2[0];
    if (hi) *hi = h2[1];
    return SPARC_OK;
}

}  // extern "C"
