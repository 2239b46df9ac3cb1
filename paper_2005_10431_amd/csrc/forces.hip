// Hellmann-Feynman atomic forces (Sec. 2: the forces used for structural
// relaxation and molecular dynamics).  At self-consistency only the explicit
// position dependence of the free energy contributes:
//   local     F_I = dV sum_x phi(x) grad b_I(x - R_I)
//                   - 1/2 dV sum over the atom's ball of grad(b_I V_I)
//   overlap   F_I = sum_{J,n}' Z_I Z_J u'(d) (R_J + nL - R_I) / d,  u(d) = erfc(d/s)/d
//   nonlocal  F_I = 2 sum_n w_n sum_k gamma_Ik (dV chi_Ik^T psi_n)(dV (grad chi_Ik)^T psi_n)
// Every sum runs over the same (grid point, periodic image) pairs as the
// corresponding energy: unwrapped grid indices inside the truncation sphere
// around the atom, wrapped to the periodic grid for field values.
// Reductions are in fixed order (no value atomics), so results are
// bitwise reproducible.
#include "internal.hpp"

namespace sg {

namespace {

constexpr double kPi = 3.14159265358979323846;

// Per-atom table: [x, y, z] * n | Z * n | rc * n | gamma (4 per atom) * n
struct ForceTab {
    const double* pos;
    const double* Z;
    const double* rc;
    const double* gamma4;
};

inline ForceTab force_tab(sparc_gpu_ctx c) {
    const int n = c->n_atoms;
    return ForceTab{c->force_tab, c->force_tab + 3 * n, c->force_tab + 4 * n, c->force_tab + 5 * n};
}

__device__ inline int wrap(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

// Fixed-order block reduction of NV values per thread (256 threads): wave
// shuffles, then the four waves in order.  Returns the block sum of value
// q = threadIdx.x for threads below NV (0 elsewhere).
template <int NV>
__device__ inline double block_reduce(const double (&v)[NV], double (*lds)[NV]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double t = v[q];
        for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
        if (lane == 0) lds[w][q] = t;
    }
    __syncthreads();
    const int q = threadIdx.x;
    return q < NV ? ((lds[0][q] + lds[1][q]) + lds[2][q]) + lds[3][q] : 0.0;
}

// Local part: block (atom, chunk of the z-range of its 8 rc box).
__global__ __launch_bounds__(256) void k_force_local(ForceTab tab, const double* __restrict__ phi, int nx, int ny,
                                                    int nz, double hx, double hy, double hz, double dV, int nchunk,
                                                    double* __restrict__ part) {
    const int a = blockIdx.x, ch = blockIdx.y;
    const double Z = tab.Z[a], rc = tab.rc[a];
    const double cx = tab.pos[3 * a], cy = tab.pos[3 * a + 1], cz = tab.pos[3 * a + 2];
    const double rmax = 8.0 * rc, rmax2 = rmax * rmax;
    const int lx = (int)ceil((cx - rmax) / hx), ux = (int)floor((cx + rmax) / hx);
    const int ly = (int)ceil((cy - rmax) / hy), uy = (int)floor((cy + rmax) / hy);
    const int lz = (int)ceil((cz - rmax) / hz), uz = (int)floor((cz + rmax) / hz);
    const int nxb = ux - lx + 1, nyb = uy - ly + 1, nzb = uz - lz + 1;
    const int z0 = lz + (int)((long)nzb * ch / nchunk), z1 = lz + (int)((long)nzb * (ch + 1) / nchunk);
    const long tot = (long)nxb * nyb * (z1 - z0);
    const double amp = -Z * pow(kPi * rc * rc, -1.5);
    const double inv = 1.0 / (rc * rc);
    double acc[3] = {0.0, 0.0, 0.0};
    for (long t = threadIdx.x; t < tot; t += blockDim.x) {
        const int i = lx + (int)(t % nxb);
        const int j = ly + (int)((t / nxb) % nyb);
        const int k = z0 + (int)(t / ((long)nxb * nyb));
        const double dx = i * hx - cx, dy = j * hy - cy, dz = k * hz - cz;
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 > rmax2) continue;
        const double ex = exp(-r2 * inv);
        const double b = amp * ex;
        const double r = sqrt(r2);
        const double V = (r < 1e-12) ? -2.0 * Z / (sqrt(kPi) * rc) : -Z * erf(r / rc) / r;
        // V'(r) / r, with its finite limit at r -> 0
        const double dVr = (r < 1e-8) ? 4.0 * Z / (3.0 * sqrt(kPi) * rc * rc * rc)
                                      : (Z * erf(r / rc) / r2 - Z * 2.0 / (sqrt(kPi) * rc) * ex / r) / r;
        const double ph = phi[wrap(i, nx) + (long)nx * (wrap(j, ny) + (long)ny * wrap(k, nz))];
        const double g = -2.0 * inv * b;    // grad b = g d
        const double s = ph * g - 0.5 * (V * g + b * dVr);
        acc[0] += s * dx;
        acc[1] += s * dy;
        acc[2] += s * dz;
    }
    __shared__ double lds[4][3];
    const double sum = block_reduce<3>(acc, lds);
    if (threadIdx.x < 3) part[((long)a * nchunk + ch) * 3 + threadIdx.x] = dV * sum;
}

// out[3 a + d] = sum over chunks (in order) of the local partials
__global__ void k_force_local_reduce(const double* __restrict__ part, int n_atoms, int nchunk,
                                     double* __restrict__ out) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3L * n_atoms) return;
    const long a = t / 3, d = t % 3;
    double s = 0.0;
    for (int ch = 0; ch < nchunk; ++ch) s += part[(a * nchunk + ch) * 3 + d];
    out[t] = s;
}

// Overlap part, added to out: one block per atom I, threads over J.
__global__ __launch_bounds__(256) void k_force_overlap(ForceTab tab, int n_atoms, double Lx, double Ly, double Lz,
                                                      double rmax, int nimx, int nimy, int nimz,
                                                      double* __restrict__ out) {
    const int I = blockIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};
    const double xI = tab.pos[3 * I], yI = tab.pos[3 * I + 1], zI = tab.pos[3 * I + 2];
    for (int J = threadIdx.x; J < n_atoms; J += blockDim.x) {
        const double s = sqrt(tab.rc[I] * tab.rc[I] + tab.rc[J] * tab.rc[J]);
        const double zz = tab.Z[I] * tab.Z[J];
        for (int a = -nimx; a <= nimx; ++a)
            for (int b = -nimy; b <= nimy; ++b)
                for (int c = -nimz; c <= nimz; ++c) {
                    if (I == J && a == 0 && b == 0 && c == 0) continue;
                    const double vx = tab.pos[3 * J] + a * Lx - xI;
                    const double vy = tab.pos[3 * J + 1] + b * Ly - yI;
                    const double vz = tab.pos[3 * J + 2] + c * Lz - zI;
                    const double d = sqrt(vx * vx + vy * vy + vz * vz);
                    if (!(d < rmax)) continue;
                    const double du = -erfc(d / s) / (d * d) - 2.0 / (sqrt(kPi) * s) * exp(-(d / s) * (d / s)) / d;
                    const double f = zz * du / d;
                    acc[0] += f * vx;
                    acc[1] += f * vy;
                    acc[2] += f * vz;
                }
    }
    __shared__ double lds[4][3];
    const double sum = block_reduce<3>(acc, lds);
    if (threadIdx.x < 3) out[3 * I + threadIdx.x] += sum;
}

// Projections of NB columns on the atom's projectors and their gradients:
// pd[(a ncol + col) 16 + q] with q = k (chi_k^T psi, k = s, px, py, pz) and
// q = 4 + 3 k + d ((d/dx_d chi_k)^T psi), each times dV.
template <typename T, int NB>
__global__ __launch_bounds__(256) void k_force_nl_proj(const T* __restrict__ X, long ldx, int ncol, ForceTab tab,
                                                      int nx, int ny, int nz, double hx, double hy, double hz,
                                                      double rc, double rcut, double N0, double N1, double dV,
                                                      double* __restrict__ pd) {
    const int a = blockIdx.x;
    const int col0 = blockIdx.y * NB;
    const double cx = tab.pos[3 * a], cy = tab.pos[3 * a + 1], cz = tab.pos[3 * a + 2];
    const double rcut2 = rcut * rcut;
    const int lx = (int)ceil((cx - rcut) / hx), ux = (int)floor((cx + rcut) / hx);
    const int ly = (int)ceil((cy - rcut) / hy), uy = (int)floor((cy + rcut) / hy);
    const int lz = (int)ceil((cz - rcut) / hz), uz = (int)floor((cz + rcut) / hz);
    const int nxb = ux - lx + 1, nyb = uy - ly + 1, nzb = uz - lz + 1;
    const long tot = (long)nxb * nyb * nzb;
    const double g = -2.0 / (rc * rc);
    double acc[NB * 16];
#pragma unroll
    for (int q = 0; q < NB * 16; ++q) acc[q] = 0.0;
    for (long t = threadIdx.x; t < tot; t += blockDim.x) {
        const int i = lx + (int)(t % nxb);
        const int j = ly + (int)((t / nxb) % nyb);
        const int k = lz + (int)(t / ((long)nxb * nyb));
        const double dx = i * hx - cx, dy = j * hy - cy, dz = k * hz - cz;
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 > rcut2) continue;
        const double e = exp(-r2 / (rc * rc));
        const double e0 = N0 * e, e1 = N1 * e;
        const double d[3] = {dx, dy, dz};
        double f[16];
        f[0] = e0;
        f[1] = e1 * dx;
        f[2] = e1 * dy;
        f[3] = e1 * dz;
#pragma unroll
        for (int b = 0; b < 3; ++b) f[4 + b] = e0 * g * d[b];
#pragma unroll
        for (int kk = 0; kk < 3; ++kk)
#pragma unroll
            for (int b = 0; b < 3; ++b) f[7 + 3 * kk + b] = e1 * ((kk == b ? 1.0 : 0.0) + g * d[kk] * d[b]);
        const long p = wrap(i, nx) + (long)nx * (wrap(j, ny) + (long)ny * wrap(k, nz));
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            if (col0 + c < ncol) {
                const double x = (double)X[p + (long)(col0 + c) * ldx];
#pragma unroll
                for (int q = 0; q < 16; ++q) acc[16 * c + q] += x * f[q];
            }
        }
    }
    __shared__ double lds[4][NB * 16];
    const double sum = block_reduce<NB * 16>(acc, lds);
    const int q = threadIdx.x;
    if (q < NB * 16) {
        const int c = q / 16;
        if (col0 + c < ncol) pd[((long)a * ncol + col0 + c) * 16 + (q % 16)] = dV * sum;
    }
}

// out[3 a + d] += 2 sum_n w_n sum_k gamma_k P_k D_kd (one block per atom;
// columns in fixed order per thread, then the fixed-order block reduction)
__global__ __launch_bounds__(256) void k_force_nl_reduce(const double* __restrict__ pd, int ncol,
                                                        const double* __restrict__ w, ForceTab tab,
                                                        double* __restrict__ out) {
    const int a = blockIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int n = threadIdx.x; n < ncol; n += blockDim.x) {
        const double* v = pd + ((long)a * ncol + n) * 16;
        for (int k = 0; k < 4; ++k) {
            const double cpk = 2.0 * tab.gamma4[4 * a + k] * w[n] * v[k];
            for (int d = 0; d < 3; ++d) acc[d] += cpk * v[4 + 3 * k + d];
        }
    }
    __shared__ double lds[4][3];
    const double sum = block_reduce<3>(acc, lds);
    if (threadIdx.x < 3) out[3 * a + threadIdx.x] += sum;
}

constexpr int kForceNB = 4;
constexpr int kLocalChunks = 8;

}  // namespace

sparc_status ensure_force_tables(sparc_gpu_ctx c) {
    if (c->force_tab) return SPARC_OK;
    const int n = c->n_atoms;
    std::vector<double> h(9 * (size_t)n, 0.0);
    for (int a = 0; a < n; ++a) {
        for (int d = 0; d < 3; ++d) h[3 * a + d] = c->pos[3 * a + d];
        h[3 * n + a] = c->Z[a];
        h[4 * n + a] = c->rc_loc[a];
        if (c->nl_lmax >= 1) {
            h[5 * n + 4 * a] = c->gamma[2 * a];
            h[5 * n + 4 * a + 1] = h[5 * n + 4 * a + 2] = h[5 * n + 4 * a + 3] = c->gamma[2 * a + 1];
        }
    }
    SG_HIP(c, hipMalloc((void**)&c->force_tab, h.size() * sizeof(double)));
    SG_HIP(c, hipMemcpyAsync(c->force_tab, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    SG_HIP(c, hipStreamSynchronize(c->stream));
    return SPARC_OK;
}

namespace {

template <typename T>
sparc_status nl_force(sparc_gpu_ctx c, const T* X, int ncol, long ldx, const double* w, double* pd, double* out) {
    const ForceTab tab = force_tab(c);
    const double rc = c->rc_nl;
    const double N0 = std::pow(2.0 / (kPi * rc * rc), 0.75);
    const double N1 = (2.0 / rc) * N0;
    dim3 grid(c->n_atoms, div_up(ncol, kForceNB));
    k_force_nl_proj<T, kForceNB><<<grid, 256, 0, c->stream>>>(X, ldx, ncol, tab, c->nx, c->ny, c->nz, c->hx, c->hy,
                                                              c->hz, rc, c->rcut_nl, N0, N1, c->dV, pd);
    k_force_nl_reduce<<<c->n_atoms, 256, 0, c->stream>>>(pd, ncol, w, tab, out);
    SG_CHECK_LAUNCH(c);
    return SPARC_OK;
}

}  // namespace

}  // namespace sg

using namespace sg;

extern "C" {

sparc_status sparc_gpu_forces(sparc_gpu_ctx c, const double* d_phi, sparc_prec prec, const void* const* d_X,
                              int n_blocks, int ncol, long ldx, const double* d_occ, double* d_forces) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    if (!d_phi || !d_forces) return set_err(c, SPARC_ERR_ARG, "forces: null potential or output");
    if (prec != SPARC_FP64 && prec != SPARC_FP32) return set_err(c, SPARC_ERR_ARG, "forces: bad precision");
    if (n_blocks < 0 || n_blocks > 2) return set_err(c, SPARC_ERR_ARG, "forces: n_blocks must be 0, 1 or 2");
    const bool nl = c->nl_lmax >= 1 && n_blocks > 0;
    if (nl) {
        if (!d_X || !d_occ) return set_err(c, SPARC_ERR_ARG, "forces: null orbital blocks or occupations");
        for (int b = 0; b < n_blocks; ++b)
            if (!d_X[b]) return set_err(c, SPARC_ERR_ARG, "forces: null orbital block");
        if (ncol < 1 || ncol > c->n_states) return set_err(c, SPARC_ERR_ARG, "forces: ncol out of range");
        if (ldx < c->nd) return set_err(c, SPARC_ERR_ARG, "forces: ldx < N_d");
    }
    sparc_status st;
    if ((st = ensure_force_tables(c)) != SPARC_OK) return st;
    const int na = c->n_atoms;
    const size_t need = std::max((size_t)na * kLocalChunks * 3, nl ? (size_t)na * ncol * 16 : 0);
    if ((st = ensure_red(c, need)) != SPARC_OK) return st;
    const ForceTab tab = force_tab(c);
    int slot = prof_begin(c, PK_FORCE_LOCAL);
    k_force_local<<<dim3(na, kLocalChunks), 256, 0, c->stream>>>(tab, d_phi, c->nx, c->ny, c->nz, c->hx, c->hy,
                                                                  c->hz, c->dV, kLocalChunks, c->red);
    k_force_local_reduce<<<div_up(3 * na, 256), 256, 0, c->stream>>>(c->red, na, kLocalChunks, d_forces);
    const double rmax = 10.0;
    k_force_overlap<<<na, 256, 0, c->stream>>>(tab, na, c->Lx, c->Ly, c->Lz, rmax, (int)std::ceil(rmax / c->Lx) + 1,
                                               (int)std::ceil(rmax / c->Ly) + 1, (int)std::ceil(rmax / c->Lz) + 1,
                                               d_forces);
    SG_CHECK_LAUNCH(c);
    prof_end(c, slot);
    if (nl) {
        slot = prof_begin(c, PK_FORCE_NL);
        for (int b = 0; b < n_blocks; ++b) {
            const double* w = d_occ + (long)b * ncol;
            if (prec == SPARC_FP64)
                st = nl_force<double>(c, (const double*)d_X[b], ncol, ldx, w, c->red, d_forces);
            else
                st = nl_force<float>(c, (const float*)d_X[b], ncol, ldx, w, c->red, d_forces);
            if (st != SPARC_OK) return st;
        }
        prof_end(c, slot);
    }
    return SPARC_OK;
}

}  // extern "C"
