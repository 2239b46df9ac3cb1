// Matrix-free Hamiltonian and the Chebyshev recurrence built on it.
//
// H x = -1/2 Delta_h x + V_eff x + sum_I sum_lm gamma_Il chi_Ilm (dV chi_Ilm^T x)
// (Sec. 2 eq. (1); matrix-free stencil and outer-product nonlocal term as in
// Sec. 2.1).  The scaled three-term Chebyshev recurrence of the CheFSI filter
// (Sec. 2.1) is fused into the epilogue of the stencil sweep, so one sweep
// streams X_k (stencil operand), X_{k-1} (recurrence term) and writes X_{k+1}
// over X_{k-1}: 3 block-sized streams per filter degree.
//
// Sweep kernel layout (one workgroup = one orbital x one y-slab x all z):
//  - the slab is `ty` full x-rows; periodic x wraps inside LDS (padded rows),
//    so only y needs halo rows, which are read from L2 (the neighbouring slabs
//    of the same orbital run on the same XCD at the same time, see the block
//    mapping below);
//  - z is marched with a register queue of 2*NO+1 planes per thread, so every
//    point of X_k is fetched from HBM once per sweep (plus 2*NO wrap planes);
//  - two LDS plane buffers alternate so one barrier per plane suffices.
#include <cmath>
#include <cstdlib>

#include "internal.hpp"

namespace sg {

template <typename T>
struct SweepArgs {
    const T* x;       // X_k, operand of H
    T* out;           // output block (may alias xprev, never x)
    const T* xprev;   // X_{k-1} or null
    long ldx;
    int nx, ny, nz;
    int ty, ntiles_y;
    StencilCoef<T> cf;
    const T* veff;
    // nonlocal part (per-slab candidate tables, see build_slab_tables)
    const uint64_t* pe8;
    const CandInfo* slab_cand;
    const int* slab_k;
    int kmax, xw, zw;
    const double* atom_pos;  // 3 n_atoms
    T inv_rc2, N0, N1, hx, hy, hz;
    const T* D;       // gamma-scaled projections, column j at D + j*ldD
    int ldD;
    const double* params;  // a, b, a0 on the device
    int mode;              // 0: H x; 1: first filter step; 2: filter step `step`
    int step;
    int ncol;
    int slab_major;        // block order: slab-major instead of orbital-major
};

// Filter coefficients of step k of the scaled recurrence:
//   e = (b-a)/2, c = (b+a)/2, sigma_1 = e/(a0-c), tau = 2/sigma_1,
//   sigma_k = 1/(tau - sigma_{k-1});
//   step 1: out = (sigma_1/e)(Hx - c x)
//   step k: out = (2 sigma_k/e)(Hx - c x) - sigma_{k-1} sigma_k xprev
__device__ inline void filter_coefs(const double* params, int mode, int step, double& alpha, double& cshift,
                                    double& beta) {
    alpha = 1.0;
    cshift = 0.0;
    beta = 0.0;
    if (mode == 0) return;
    double A = params[0], B = params[1], A0 = params[2];
    double e = 0.5 * (B - A), c = 0.5 * (B + A);
    double s1 = e / (A0 - c);
    cshift = c;
    if (mode == 1) {
        alpha = s1 / e;
        return;
    }
    double tau = 2.0 / s1;
    double sp = s1, s = s1;
    for (int k = 2; k <= step; ++k) {
        sp = s;
        s = 1.0 / (tau - s);
    }
    alpha = 2.0 * s / e;
    beta = -sp * s;
}

constexpr int RING = 2 * kMaxHalfOrder + 2;  // z-queue slots (one spare for prefetch)

// Per-thread registers of the sweep: the z-queue ring (plane z lives in slot
// z mod RING), the prefetched halo values of the next plane, and the next
// plane's X_{k-1} and V_eff values.  Indices are compile-time after
// unrolling, so everything stays in VGPRs.
template <typename T, int HM>
struct SweepRegs {
    T q[RING];
    T h[HM];             // next plane's halo values (this thread's share)
    T xp[2];
    T ve[2];
    uint64_t pe8[2];     // own point's projector candidates (bytes, 0xFF pads)
};

template <typename T>
struct SweepGeom {
    const void* xc;
    void* oc;
    const void* pc;
    long plane, pxy;
    int nz, col, hn;
    bool active;
    int goff[6], loff[6], poff[6];  // per halo value of this thread (HM <= 6 used)
    int lrow;  // LDS offset of this thread's own point
    int W, nx, lx, ly, gy, t, nt;
    // LDS tables of the slab's projector candidates (K of them):
    T* delta;               // x offset of the candidate's first ex entry from its centre
    T* cz;                  // image-shifted z centre
    int* cxb;               // x index of the candidate's first ex entry (grid row coordinates)
    T* ex;                  // ex[k*xw + i]: exp(-dx^2/rc^2) over the candidate's x-range
    T* ez;                  // ez[k*zw + i]: exp(-dz^2/rc^2) over the candidate's z-range
    int* czb;               // z index offset into the ez table
    T* F;                   // F[(row*K + k)*3 + {0,1,2}]: z-independent factors (see sweep_ab)
    T* ab;                  // ab[parity][row][k][2]: A', B' of plane z / z+1
    int K, y0, tyn, xw, zw;
    int abk0, abdk;  // candidate of this thread's first sweep_ab pair, and its step per nt pairs
};

// A'(row, k), B'(row, k) of one plane z.  The candidate's contribution at
// a point of the row is ex(x) (A + B dx) with
//   A = ey ez (N0 D_s + N1 (dy D_py + dz D_pz)),  B = ey ez N1 D_px;
// the z-independent factors F0 = ey (N0 D_s + N1 dy D_py), F1 = ey N1 D_pz,
// F2 = ey N1 D_px are tabulated once per workgroup, so A = ez (F0 + F1 dz),
// B = ez F2.  With dx = delta_k + hx i (i the point's index in the ex table)
// the apply needs A' = A + B delta_k and B' = B hx.
template <typename T>
__device__ __forceinline__ void sweep_ab(const SweepArgs<T>& a, const SweepGeom<T>& g, int z, T* abz) {
    const int n = g.tyn * g.K;
    const T zh = (T)z * a.hz;
    int k = g.abk0;  // candidate of pair j = row * K + k
    for (int j = g.t; j < n; j += g.nt) {
        // planes outside the candidate's z-range never reach a point that
        // lists it; clamp the table index there
        const int iz = min(max(z - g.czb[k], 0), g.zw - 1);
        const T E = g.ez[k * g.zw + iz];
        const T dz = zh - g.cz[k];
        const T* F = g.F + 3 * j;
        const T A = E * (F[0] + F[1] * dz);
        const T B = E * F[2];
        abz[2 * j] = A + B * g.delta[k];
        abz[2 * j + 1] = B * a.hx;
        k += g.abdk;  // abdk = nt mod K
        if (k >= g.K) k -= g.K;
    }
}



// One z-plane of the sweep at ring phase U (z = z0 + U).  On entry the LDS
// buffer of parity U holds plane z (own rows with x-wrap padding, halo rows,
// and the plane's projector entries), written during the previous step.
//  1. barrier,
//  2. issue the loads of plane z+1 (halo rows, projector entries, own
//     X_{k-1}, V_eff and entry range; the plane index wraps so the loads are
//     unconditional and the step is straight-line code),
//  3. stencil + potential + nonlocal + recurrence for plane z, store,
//  4. write plane z+1 into the other LDS buffer (its loads have had the
//     whole compute phase to land),
//  5. load plane z + NO + 2 into the ring slot freed by plane z - NO.
// Threads without a point of the slab (ragged slab, padding to 64) load
// valid clamped addresses and compute on them, but never store.
template <int U, typename T, bool NL, int MODE, int HM>
__device__ __forceinline__ void sweep_step(const SweepArgs<T>& a, SweepRegs<T, HM>& r, const SweepGeom<T>& g,
                                           T* buf0, T* buf1, int z, T alpha, T cshift, T beta) {
    constexpr int NO = kMaxHalfOrder;
    constexpr int P = U & 1, PN = (U + 1) & 1;
    constexpr int C = U % RING;
    const T* __restrict__ xc = (const T*)g.xc;
    __syncthreads();
    const int z1 = (z + 1 == g.nz) ? 0 : z + 1;
    const long zoff1 = (long)z1 * g.plane;
#pragma unroll
    for (int i = 0; i < HM; ++i) r.h[i] = xc[g.goff[i] + zoff1];
    if (MODE == 2) r.xp[PN] = ((const T*)g.pc)[g.pxy + zoff1];
    r.ve[PN] = a.veff[g.pxy + zoff1];
    if (NL) r.pe8[PN] = a.pe8[g.pxy + zoff1];

    T* buf = P ? buf1 : buf0;
    const T* rp = buf + g.lrow;
    const int W = g.W;
    T lap = a.cf.c0 * r.q[C];
#pragma unroll
    for (int k = 1; k <= NO; ++k) lap += a.cf.cz[k] * (r.q[(U + k) % RING] + r.q[(U + RING - k) % RING]);
#pragma unroll
    for (int k = 1; k <= NO; ++k) lap += a.cf.cx[k] * (rp[k] + rp[-k]);
#pragma unroll
    for (int k = 1; k <= NO; ++k) lap += a.cf.cy[k] * (rp[k * W] + rp[-k * W]);
    const long p = g.pxy + (long)z * g.plane;
    T hv = lap + r.ve[P] * r.q[C];
    if (NL) {
        // sum over the projectors whose support holds this point of
        // chi_s D_s + chi_p . D_p = ex(x) (A + B dx)   (see sweep_ab)
        const T* abr = g.ab + (P * a.ty + (g.active ? g.ly : 0)) * 2 * g.K;
        uint64_t w = g.active ? r.pe8[P] : ~0ull;
        T nl = 0;
        for (int j = 0; j < 7; ++j) {
            const int k = (int)(w & 0xFFull);
            if (k == 0xFF) break;
            w >>= 8;
            const int i = g.lx - g.cxb[k];
            nl += g.ex[k * g.xw + i] * (abr[2 * k] + abr[2 * k + 1] * (T)i);
        }
        hv += nl;
    }
    T o;
    if (MODE == 0) {
        o = hv;
    } else {
        o = alpha * (hv - cshift * r.q[C]);
        if (MODE == 2) o += beta * r.xp[P];
    }
    if (g.active) ((T*)g.oc)[p] = o;

    // plane z+1 into the other buffer
    T* nbuf = P ? buf0 : buf1;
    constexpr int CN = (U + 1) % RING;
    if (g.active) {
        nbuf[g.lrow] = r.q[CN];
        if (g.lx < NO) nbuf[g.lrow + g.nx] = r.q[CN];
        if (g.lx >= g.nx - NO) nbuf[g.lrow - g.nx] = r.q[CN];
    }
#pragma unroll
    for (int i = 0; i < HM; ++i)
        if (i < g.hn) {
            nbuf[g.loff[i]] = r.h[i];
            if (g.poff[i] >= 0) nbuf[g.poff[i]] = r.h[i];
        }
    if (NL) sweep_ab<T>(a, g, z1, g.ab + PN * a.ty * 2 * g.K);  // A/B of the next plane
    int zn = z + NO + 2;
    zn = zn >= g.nz ? zn - g.nz : zn;
    r.q[(U + NO + 2) % RING] = xc[g.pxy + (long)zn * g.plane];
}

// Workgroups of the nonlocal variant are capped at 512 threads so that its
// extra live registers (entry prefetch, projector evaluation) fit without
// spilling.
template <typename T, bool NL, int MODE, int HM>
__global__ __attribute__((amdgpu_flat_work_group_size(1, NL ? 512 : 1024))) void k_hsweep(SweepArgs<T> a) {
    constexpr int NO = kMaxHalfOrder;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* buf0 = reinterpret_cast<T*>(smem_raw);
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int W = nx + 2 * NO;
    const int R = a.ty + 2 * NO;
    T* buf1 = buf0 + R * W;

    // Hardware dispatches block b to XCD b % 8.  Give each XCD a contiguous
    // range of logical tiles so that the y-slabs of one orbital (which read
    // each other's rows as halos) share an L2.
    const int nblk = gridDim.x, bid = blockIdx.x;
    const int qn = nblk / 8, rn = nblk % 8;
    const int xcd = bid % 8, slot = bid / 8;
    const int logical = xcd * qn + min(xcd, rn) + slot;
    int col, tile;
    if (a.slab_major) {
        // all orbitals of one slab back to back: the slab's projector
        // entries stay resident in the XCD's L2
        tile = logical / a.ncol;
        col = logical - tile * a.ncol;
    } else {
        col = logical / a.ntiles_y;
        tile = logical - col * a.ntiles_y;
    }
    const int y0 = tile * a.ty;
    const int tyn = min(a.ty, ny - y0);

    const int t = threadIdx.x;
    const int nt = blockDim.x;
    const int lx = t % nx, ly = t / nx;

    SweepGeom<T> g;
    g.active = ly < tyn;
    g.plane = (long)nx * ny;
    g.nz = nz;
    g.col = col;
    g.W = W;
    g.nx = nx;
    g.lx = lx;
    g.gy = y0 + (g.active ? ly : 0);
    g.ly = ly;
    g.t = t;
    g.nt = nt;
    g.y0 = y0;
    g.tyn = tyn;
    if (NL) {
        // LDS after the two plane buffers (layout of nl_sweep_lds_bytes):
        // delta, cz (K T each), ex (K xw), ez (K zw), F (3 ty K), A'/B'
        // (2 planes x 2 ty K), cxb, czb (K int each)
        const int KM = a.kmax;
        T* tp = buf1 + R * W;
        g.delta = tp;
        g.cz = tp + KM;
        g.ex = tp + 2 * KM;
        g.ez = g.ex + KM * a.xw;
        g.F = g.ez + KM * a.zw;
        g.ab = g.F + 3 * a.ty * KM;
        g.cxb = reinterpret_cast<int*>(g.ab + 4 * a.ty * KM);
        g.czb = g.cxb + KM;
        g.xw = a.xw;
        g.zw = a.zw;
        g.K = a.slab_k[tile];
        g.abk0 = g.K > 0 ? t % g.K : 0;
        g.abdk = g.K > 0 ? nt % g.K : 0;
        const CandInfo* ci = a.slab_cand + (long)tile * KM;
        const T* Dc = a.D + (long)col * a.ldD;
        for (int k = t; k < g.K; k += nt) {
            const CandInfo c = ci[k];
            g.delta[k] = (T)((double)c.ixlo * (double)a.hx - a.atom_pos[3 * c.atom]);
            g.cz[k] = (T)(a.atom_pos[3 * c.atom + 2] - (double)c.sz * (double)nz * (double)a.hz);
            g.cxb[k] = c.ixlo - c.sx * nx;
            g.czb[k] = c.izlo - c.sz * nz;
        }
        for (int j = t; j < g.K * g.xw; j += nt) {
            const int k = j / g.xw, i = j - k * g.xw;
            const T dx = (T)(ci[k].ixlo + i) * a.hx - (T)a.atom_pos[3 * ci[k].atom];
            g.ex[j] = exp(-dx * dx * a.inv_rc2);
        }
        for (int j = t; j < g.K * g.zw; j += nt) {
            const int k = j / g.zw, i = j - k * g.zw;
            const T dz = (T)(ci[k].izlo + i) * a.hz - (T)a.atom_pos[3 * ci[k].atom + 2];
            g.ez[j] = exp(-dz * dz * a.inv_rc2);
        }
        for (int j = t; j < tyn * g.K; j += nt) {
            const int row = j / g.K, k = j - row * g.K;
            const CandInfo c = ci[k];
            const T cy = (T)(a.atom_pos[3 * c.atom + 1] - (double)c.sy * (double)ny * (double)a.hy);
            const T dy = (T)(y0 + row) * a.hy - cy;
            const T ey = exp(-dy * dy * a.inv_rc2);
            const T* Dk = Dc + 4 * c.atom;
            g.F[3 * j] = ey * (a.N0 * Dk[0] + a.N1 * dy * Dk[2]);
            g.F[3 * j + 1] = ey * a.N1 * Dk[3];
            g.F[3 * j + 2] = ey * a.N1 * Dk[1];
        }
        __syncthreads();
        sweep_ab<T>(a, g, 0, g.ab);
    }
    const T* xc = a.x + (long)col * a.ldx;
    g.xc = xc;
    g.oc = a.out + (long)col * a.ldx;
    g.pc = a.xprev ? a.xprev + (long)col * a.ldx : nullptr;
    g.pxy = lx + (long)nx * (y0 + (g.active ? ly : 0));
    g.lrow = (ly + NO) * W + NO + lx;
    // halo rows: 2 NO rows of nx values per plane, spread over the threads
    const int nhalo = 2 * NO * nx;
    g.hn = 0;
#pragma unroll
    for (int i = 0; i < HM; ++i) {
        const int e = t + i * nt;
        g.goff[i] = 0;
        g.loff[i] = 0;
        g.poff[i] = -1;
        if (e < nhalo) {
            g.hn = i + 1;
            int hr = e / nx, hx = e - hr * nx;
            int lrow, gy;
            if (hr < NO) {
                lrow = hr;
                gy = y0 - NO + hr;
            } else {
                lrow = NO + tyn + (hr - NO);
                gy = y0 + tyn + (hr - NO);
            }
            gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
            g.goff[i] = hx + nx * gy;
            g.loff[i] = lrow * W + NO + hx;
            if (hx < NO) g.poff[i] = g.loff[i] + nx;
            if (hx >= nx - NO) g.poff[i] = g.loff[i] - nx;
        }
    }

    double alpha_d, c_d, beta_d;
    filter_coefs(a.params, MODE, a.step, alpha_d, c_d, beta_d);
    const T alpha = (T)alpha_d, cshift = (T)c_d, beta = (T)beta_d;

    SweepRegs<T, HM> r;
    // ring: planes -NO .. NO+1 (slot = plane mod RING), plane 0 prefetches
#pragma unroll
    for (int j = -NO; j <= NO + 1; ++j) {
        int zz = j < 0 ? j + nz : j;
        r.q[(j + RING) % RING] = xc[g.pxy + (long)zz * g.plane];
    }
    r.xp[0] = (MODE == 2) ? ((const T*)g.pc)[g.pxy] : (T)0;
    r.ve[0] = a.veff[g.pxy];
    // plane 0 into LDS buffer 0
    if (g.active) {
        buf0[g.lrow] = r.q[0];
        if (lx < NO) buf0[g.lrow + nx] = r.q[0];
        if (lx >= nx - NO) buf0[g.lrow - nx] = r.q[0];
    }
#pragma unroll
    for (int i = 0; i < HM; ++i)
        if (i < g.hn) {
            T v = xc[g.goff[i]];
            buf0[g.loff[i]] = v;
            if (g.poff[i] >= 0) buf0[g.poff[i]] = v;
        }
    if (NL) r.pe8[0] = a.pe8[g.pxy];

#define SG_STEP(U)                                                                     \
    if (z0 + U >= nz) break;                                                           \
    sweep_step<U, T, NL, MODE, HM>(a, r, g, buf0, buf1, z0 + U, alpha, cshift, beta);
    for (int z0 = 0; z0 < nz; z0 += RING) {
        SG_STEP(0) SG_STEP(1) SG_STEP(2) SG_STEP(3) SG_STEP(4) SG_STEP(5) SG_STEP(6)
        SG_STEP(7) SG_STEP(8) SG_STEP(9) SG_STEP(10) SG_STEP(11) SG_STEP(12) SG_STEP(13)
    }
#undef SG_STEP
}

// D(4a+lm, j) = gamma_lm * dV * sum over the image points p of atom a's
// ball of chi_lm(p) X(idx(p), j), accumulated in double in a fixed order
// (deterministic).  chi_s = N0 e, chi_p = N1 {dx, dy, dz} e with
// e = ex(x) ey(y) ez(z) from per-axis tables of the atom's bounding box,
// evaluated in LDS (no per-point projector table is read).
template <typename T, int NB, int U>
__global__ __launch_bounds__(256) void k_projection(const T* __restrict__ x, long ldx, int ncol,
                                                    const long* __restrict__ ip_off, const int* __restrict__ ip_idx,
                                                    const uint32_t* __restrict__ ip_box, const int* __restrict__ box_lo,
                                                    int ext, const double* __restrict__ pos, double hx, double hy,
                                                    double hz, double inv_rc2, double N0, double N1,
                                                    const double* __restrict__ g4, double dV, T* __restrict__ D,
                                                    int ldD, const int* __restrict__ atom_order, int n_atoms) {
    // Block b runs on XCD b % 8.  Atoms are visited in a space-filling order
    // and each XCD takes a contiguous range of it for one orbital chunk at a
    // time, so overlapping supports of neighbouring atoms hit in that XCD's L2.
    extern __shared__ double ptab[];  // e and d tables: ex, ey, ez, dx, dy, dz (ext each)
    const int bid = blockIdx.x;
    const int xcd = bid % 8, slot = bid / 8;
    const int per = (n_atoms + 7) / 8;
    const int rank = xcd * per + slot % per;
    const int chunk = slot / per;
    if (rank >= n_atoms || chunk * NB >= ncol) return;
    const int a = atom_order[rank];
    for (int q = threadIdx.x; q < 3 * ext; q += blockDim.x) {
        const int d = q / ext, i = q - d * ext;
        const double h = d == 0 ? hx : (d == 1 ? hy : hz);
        const double dv = (double)(box_lo[3 * a + d] + i) * h - pos[3 * a + d];
        ptab[q] = exp(-dv * dv * inv_rc2);
        ptab[3 * ext + q] = dv;
    }
    __syncthreads();
    const double* ex = ptab;
    const double* ey = ptab + ext;
    const double* ez = ptab + 2 * ext;
    const double* dxt = ptab + 3 * ext;
    const double* dyt = ptab + 4 * ext;
    const double* dzt = ptab + 5 * ext;
    const int n0 = chunk * NB;
    const int nb = min(NB, ncol - n0);
    double acc[NB][4];
#pragma unroll
    for (int n = 0; n < NB; ++n)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[n][k] = 0.0;
    // U points per thread are in flight at once: their indices, then their
    // X values, are loaded before any is accumulated (each thread still
    // accumulates its points s0 + t, s0 + t + nt, ... in increasing order).
    const long s0 = ip_off[a], s1 = ip_off[a + 1];
    const int nt = blockDim.x;
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
        double v[U][NB];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int n = 0; n < NB; ++n)
                v[u][n] = (bb[u] != 0xFFFFFFFFu && n < nb) ? (double)x[idx[u] + (long)(n0 + n) * ldx] : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (bb[u] == 0xFFFFFFFFu) break;
            const uint32_t b = bb[u];
            const int bx = b & 0xFF, by = (b >> 8) & 0xFF, bz = (b >> 16) & 0xFF;
            const double e = ex[bx] * ey[by] * ez[bz];
            const double c0 = N0 * e, c1 = N1 * dxt[bx] * e, c2 = N1 * dyt[by] * e, c3 = N1 * dzt[bz] * e;
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                if (n < nb) {
                    acc[n][0] += c0 * v[u][n];
                    acc[n][1] += c1 * v[u][n];
                    acc[n][2] += c2 * v[u][n];
                    acc[n][3] += c3 * v[u][n];
                }
            }
        }
    }
    // wave reduction then across the 4 waves
    __shared__ double part[4][NB * 4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int n = 0; n < NB; ++n)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            double v = acc[n][k];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
            if (lane == 0) part[wv][n * 4 + k] = v;
        }
    __syncthreads();
    if (threadIdx.x < NB * 4) {
        int n = threadIdx.x / 4, k = threadIdx.x % 4;
        if (n < nb) {
            double v = ((part[0][threadIdx.x] + part[1][threadIdx.x]) + part[2][threadIdx.x]) + part[3][threadIdx.x];
            D[(long)(n0 + n) * ldD + 4 * a + k] = (T)(g4[4 * a + k] * dV * v);
        }
    }
}

int choose_sweep_ty(int nx, int ny, int max_threads) {
    // tuning override: rows per y-slab
    if (const char* e = std::getenv("SPARC_GPU_SWEEP_TY")) {
        int v = std::atoi(e);
        if (v >= 2 && v <= ny && ((v * nx + 63) / 64) * 64 <= max_threads) return v;
    }
    int maxty = std::max(1, std::min(16, max_threads / nx));
    maxty = std::min(maxty, ny);
    // prefer the largest divisor of ny not above maxty, unless it is small
    int best = 1;
    for (int t = maxty; t >= 1; --t)
        if (ny % t == 0) {
            best = t;
            break;
        }
    if (best * 2 < maxty) best = maxty;
    return best;
}

template <typename T>
static const StencilCoef<T>& coef(sparc_gpu_ctx c);
template <>
const StencilCoef<double>& coef<double>(sparc_gpu_ctx c) {
    return c->cf64;
}
template <>
const StencilCoef<float>& coef<float>(sparc_gpu_ctx c) {
    return c->cf32;
}

template <typename T>
static const T* veff_of(sparc_gpu_ctx c);
template <>
const double* veff_of<double>(sparc_gpu_ctx c) {
    return c->veff;
}
template <>
const float* veff_of<float>(sparc_gpu_ctx c) {
    return c->veff32;
}

template <typename T>
static T* D_of(sparc_gpu_ctx c);
template <>
double* D_of<double>(sparc_gpu_ctx c) {
    return c->D;
}
template <>
float* D_of<float>(sparc_gpu_ctx c) {
    return c->D32;
}

template <typename T>
sparc_status launch_hsweep(sparc_gpu_ctx c, const T* x, T* out, const T* xprev, int ncol, long ldx, int mode,
                           int step, int dcol0, hipStream_t s) {
    hipStream_t stream = s ? s : c->stream;
    SweepArgs<T> a;
    a.x = x;
    a.out = out;
    a.xprev = xprev;
    a.ldx = ldx;
    a.nx = c->nx;
    a.ny = c->ny;
    a.nz = c->nz;
    a.ty = choose_sweep_ty(c->nx, c->ny, 1024);
    a.ntiles_y = div_up(c->ny, a.ty);
    a.cf = coef<T>(c);
    a.veff = veff_of<T>(c);
    const bool nl = !c->sweep_local_only && c->nl_lmax >= 1 && c->nl.n_pe > 0;
    if (nl) {
        a.ty = c->nl_ty;
        a.ntiles_y = div_up(c->ny, a.ty);
    }
    a.pe8 = c->nl.pe8;
    a.slab_cand = c->nl.slab_cand;
    a.slab_k = c->nl.slab_k;
    a.kmax = c->nl.slab_kmax;
    a.xw = c->nl.slab_xw;
    a.zw = c->nl.slab_zw;
    a.atom_pos = c->atom_pos;
    {
        const double pi = 3.14159265358979323846;
        const double rc = c->rc_nl > 0 ? c->rc_nl : 1.0;
        const double N0 = std::pow(2.0 / (pi * rc * rc), 0.75);
        a.inv_rc2 = (T)(1.0 / (rc * rc));
        a.N0 = (T)N0;
        a.N1 = (T)((2.0 / rc) * N0);
        a.hx = (T)c->hx;
        a.hy = (T)c->hy;
        a.hz = (T)c->hz;
    }
    a.D = D_of<T>(c) + (long)dcol0 * 4 * c->n_atoms;
    a.ldD = 4 * c->n_atoms;
    a.params = c->scal + S_A;
    a.mode = mode;
    a.step = step;
    a.ncol = ncol;
    a.slab_major = c->sweep_slab_major;
    const int threads = div_up((long)c->nx * a.ty, 64) * 64;
    size_t shmem = 2 * (size_t)(a.ty + 2 * kMaxHalfOrder) * (c->nx + 2 * kMaxHalfOrder) * sizeof(T);
    if (nl) shmem = nl_sweep_lds_bytes(a.ty, c->nx, a.kmax, a.xw, a.zw, sizeof(T));
    if (shmem > 160 * 1024) return set_err(c, SPARC_ERR_ARG, "sweep workgroup needs more than 160 KB of LDS");
    if (threads > (nl ? 512 : 1024)) return set_err(c, SPARC_ERR_ARG, "grid x-extent too large for the sweep kernel");
    const long nblocks = (long)ncol * a.ntiles_y;
    if (nblocks > 0x7fffffffL) return set_err(c, SPARC_ERR_ARG, "too many blocks");
    const int hm = div_up(2L * kMaxHalfOrder * c->nx, threads);
    if (hm > (nl ? 6 : 3)) return set_err(c, SPARC_ERR_ARG, "grid x-extent too large for the sweep kernel");
    const int slot = prof_begin(c, mode == 2 ? PK_SWEEP : (mode == 1 ? PK_SWEEP1 : PK_APPLY), stream);
    const dim3 g((unsigned)nblocks), b(threads);
#define SG_LAUNCH_SWEEP(NLV, MV, HMV) k_hsweep<T, NLV, MV, HMV><<<g, b, shmem, stream>>>(a)
#define SG_SWEEP_HM(NLV, MV)          \
    do {                              \
        if (hm == 1) SG_LAUNCH_SWEEP(NLV, MV, 1); \
        else if (hm == 2) SG_LAUNCH_SWEEP(NLV, MV, 2); \
        else SG_LAUNCH_SWEEP(NLV, MV, 3); \
    } while (0)
    // the nonlocal variant's slab can be as low as 2 rows on wide grids
    // (its candidate tables share the LDS), hence up to 6 halo values
#define SG_SWEEP_HM_NL(MV)            \
    do {                              \
        if (hm <= 3) SG_SWEEP_HM(true, MV); \
        else if (hm == 4) SG_LAUNCH_SWEEP(true, MV, 4); \
        else if (hm == 5) SG_LAUNCH_SWEEP(true, MV, 5); \
        else SG_LAUNCH_SWEEP(true, MV, 6); \
    } while (0)
    if (nl) {
        if (mode == 0) SG_SWEEP_HM_NL(0);
        else if (mode == 1) SG_SWEEP_HM_NL(1);
        else SG_SWEEP_HM_NL(2);
    } else {
        if (mode == 0) SG_SWEEP_HM(false, 0);
        else if (mode == 1) SG_SWEEP_HM(false, 1);
        else SG_SWEEP_HM(false, 2);
    }
#undef SG_SWEEP_HM_NL
#undef SG_SWEEP_HM
#undef SG_LAUNCH_SWEEP
    SG_CHECK_LAUNCH(c);
    prof_end(c, slot, stream);
    return SPARC_OK;
}

template <typename T>
sparc_status launch_projection(sparc_gpu_ctx c, const T* x, int ncol, long ldx, int dcol0, hipStream_t s) {
    if (c->nl_lmax < 1 || c->nl.n_sup == 0) return SPARC_OK;
    hipStream_t stream = s ? s : c->stream;
    const int per = (c->n_atoms + 7) / 8;
    const int slot = prof_begin(c, PK_PROJ, stream);
    const double pi = 3.14159265358979323846;
    const double rc = c->rc_nl;
    const double N0 = std::pow(2.0 / (pi * rc * rc), 0.75), N1 = (2.0 / rc) * N0;
    const int ext = c->nl.box_ext;
    T* Dd = D_of<T>(c) + (long)dcol0 * 4 * c->n_atoms;
#define SG_PROJ(NBV, UV)                                                                                           \
    k_projection<T, NBV, UV><<<dim3(8 * per * div_up(ncol, NBV)), 256, 6 * ext * sizeof(double), stream>>>(            \
        x, ldx, ncol, c->nl.ip_off, c->nl.ip_idx, c->nl.ip_box, c->nl.box_lo, ext, c->atom_pos, c->hx, c->hy, c->hz, \
        1.0 / (rc * rc), N0, N1, c->nl.gamma4, c->dV, Dd, 4 * c->n_atoms, c->nl.atom_order, c->n_atoms)
    // columns per workgroup (tuning override SPARC_GPU_PROJ_NB = 2, 4 or 8):
    // fewer accumulators per thread keep more waves in flight for the gather
    // and points in flight per thread (SPARC_GPU_PROJ_U = 1, 2 or 4; by
    // default 2 in FP64 and 1 in FP32, the faster of each on cfg2)
    const int pu = c->proj_u > 0 ? c->proj_u : (sizeof(T) == 8 ? 2 : 1);
    if (c->proj_nb == 2)
        SG_PROJ(2, 4);
    else if (c->proj_nb == 8)
        SG_PROJ(8, 2);
    else if (pu == 1)
        SG_PROJ(4, 1);
    else if (pu == 4)
        SG_PROJ(4, 4);
    else
        SG_PROJ(4, 2);
#undef SG_PROJ
    SG_CHECK_LAUNCH(c);
    prof_end(c, slot, stream);
    return SPARC_OK;
}

template sparc_status launch_hsweep<double>(sparc_gpu_ctx, const double*, double*, const double*, int, long, int,
                                            int, int, hipStream_t);
template sparc_status launch_hsweep<float>(sparc_gpu_ctx, const float*, float*, const float*, int, long, int, int,
                                           int, hipStream_t);
template sparc_status launch_projection<double>(sparc_gpu_ctx, const double*, int, long, int, hipStream_t);
template sparc_status launch_projection<float>(sparc_gpu_ctx, const float*, int, long, int, hipStream_t);

template <typename T>
static sparc_status apply_impl(sparc_gpu_ctx c, const T* X, T* Y, int ncol, long ldx) {
    sparc_status st = launch_projection<T>(c, X, ncol, ldx);
    if (st != SPARC_OK) return st;
    return launch_hsweep<T>(c, X, Y, nullptr, ncol, ldx, 0, 0);
}

template <typename T>
__global__ void k_copy_block(const T* __restrict__ src, T* __restrict__ dst, long nd, int ncol, long ld) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    if (i < nd && j < ncol) dst[i + (long)j * ld] = src[i + (long)j * ld];
}

// Filter with bounds already in c->scal[S_A..S_A0].  Y_k lives in X when k is
// even and in W when k is odd; the result ends in X.
//
// One chain of the filter over columns [col0, col0 + ncol) on stream s.
template <typename T>
static sparc_status filter_chain(sparc_gpu_ctx c, T* X, T* Wk, int col0, int ncol, long ldx, int m, hipStream_t s) {
    sparc_status st;
    X += (long)col0 * ldx;
    Wk += (long)col0 * ldx;
    if ((st = launch_projection<T>(c, X, ncol, ldx, col0, s)) != SPARC_OK) return st;
    if ((st = launch_hsweep<T>(c, X, Wk, nullptr, ncol, ldx, 1, 1, col0, s)) != SPARC_OK) return st;
    for (int k = 2; k <= m; ++k) {
        T* cur = (k % 2 == 0) ? Wk : X;   // Y_{k-1}
        T* dst = (k % 2 == 0) ? X : Wk;   // Y_{k-2}, overwritten with Y_k
        if ((st = launch_projection<T>(c, cur, ncol, ldx, col0, s)) != SPARC_OK) return st;
        if ((st = launch_hsweep<T>(c, cur, dst, dst, ncol, ldx, 2, k, col0, s)) != SPARC_OK) return st;
    }
    if (m % 2 == 1) {
        dim3 grid(div_up(c->nd, 256), ncol);
        k_copy_block<T><<<grid, 256, 0, s>>>(Wk, X, c->nd, ncol, ldx);
        SG_CHECK_LAUNCH(c);
    }
    return SPARC_OK;
}

// The filter acts on every column independently.  Optionally (context flag
// split_filter, off by default) a block of at least 64 columns with
// projectors is split in two halves filtered on two streams, the second
// started one projection later, so that kernels of the two halves overlap.
// The default is one stream: concurrent halves make the per-launch times
// of the sweep overlap each other.
template <typename T>
sparc_status filter_impl(sparc_gpu_ctx c, T* X, T* Wk, int ncol, long ldx, int m) {
    const bool nl = c->nl_lmax >= 1 && c->nl.n_sup > 0;
    if (!nl || ncol < 64 || !c->split_filter) return filter_chain<T>(c, X, Wk, 0, ncol, ldx, m, c->stream);
    if (!c->aux_stream) {
        SG_HIP(c, hipStreamCreateWithFlags(&c->aux_stream, hipStreamNonBlocking));
        SG_HIP(c, hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
        SG_HIP(c, hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming));
    }
    const int na = ncol / 2, nb = ncol - na;
    sparc_status st;
    // second half: starts after the first half's first projection (and after
    // everything queued before this call on the context stream)
    if ((st = launch_projection<T>(c, X, na, ldx, 0, c->stream)) != SPARC_OK) return st;
    SG_HIP(c, hipEventRecord(c->fork_ev, c->stream));
    SG_HIP(c, hipStreamWaitEvent(c->aux_stream, c->fork_ev, 0));
    if ((st = filter_chain<T>(c, X, Wk, na, nb, ldx, m, c->aux_stream)) != SPARC_OK) return st;
    // first half (its first projection is already queued)
    if ((st = launch_hsweep<T>(c, X, Wk, nullptr, na, ldx, 1, 1, 0, c->stream)) != SPARC_OK) return st;
    for (int k = 2; k <= m; ++k) {
        T* cur = (k % 2 == 0) ? Wk : X;
        T* dst = (k % 2 == 0) ? X : Wk;
        if ((st = launch_projection<T>(c, cur, na, ldx, 0, c->stream)) != SPARC_OK) return st;
        if ((st = launch_hsweep<T>(c, cur, dst, dst, na, ldx, 2, k, 0, c->stream)) != SPARC_OK) return st;
    }
    if (m % 2 == 1) {
        dim3 grid(div_up(c->nd, 256), na);
        k_copy_block<T><<<grid, 256, 0, c->stream>>>(Wk, X, c->nd, na, ldx);
        SG_CHECK_LAUNCH(c);
    }
    SG_HIP(c, hipEventRecord(c->join_ev, c->aux_stream));
    SG_HIP(c, hipStreamWaitEvent(c->stream, c->join_ev, 0));
    return SPARC_OK;
}

template sparc_status filter_impl<double>(sparc_gpu_ctx, double*, double*, int, long, int);
template sparc_status filter_impl<float>(sparc_gpu_ctx, float*, float*, int, long, int);

__global__ void k_set3(double* dst, double a, double b, double c) {
    dst[0] = a;
    dst[1] = b;
    dst[2] = c;
}

__global__ void k_veff_convert(const double* src, double* dst, float* dst32, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        double v = src[i];
        dst[i] = v;
        dst32[i] = (float)v;
    }
}

sparc_status set_veff_impl(sparc_gpu_ctx c, const double* d_veff) {
    if (d_veff != c->veff) {
        k_veff_convert<<<div_up(c->nd, 256), 256, 0, c->stream>>>(d_veff, c->veff, c->veff32, c->nd);
    } else {
        k_veff_convert<<<div_up(c->nd, 256), 256, 0, c->stream>>>(c->veff, c->veff, c->veff32, c->nd);
    }
    SG_CHECK_LAUNCH(c);
    return SPARC_OK;
}

// lo = min V_eff + nl_lo, hi = kin + max V_eff + nl_hi
// Extrema of V_eff: per-block partials (part[2 b], part[2 b + 1]), then one
// block combines them into the spectrum bounds.
__global__ __launch_bounds__(256) void k_minmax_part(const double* v, long n, double* part) {
    __shared__ double smin[256], smax[256];
    double mn = 1e300, mx = -1e300;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double x = v[i];
        mn = fmin(mn, x);
        mx = fmax(mx, x);
    }
    smin[threadIdx.x] = mn;
    smax[threadIdx.x] = mx;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = smin[0];
        part[2 * blockIdx.x + 1] = smax[0];
    }
}

__global__ __launch_bounds__(256) void k_bounds(const double* part, int nblk, double kin, double nl_lo,
                                                double nl_hi, double* out_lo, double* out_hi) {
    __shared__ double smin[256], smax[256];
    double mn = 1e300, mx = -1e300;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
        mn = fmin(mn, part[2 * b]);
        mx = fmax(mx, part[2 * b + 1]);
    }
    smin[threadIdx.x] = mn;
    smax[threadIdx.x] = mx;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *out_lo = smin[0] + nl_lo;
        *out_hi = kin + smax[0] + nl_hi;
    }
}

sparc_status bounds_impl(sparc_gpu_ctx c) {
    const int nblk = (int)std::min<long>(512, div_up(c->nd, 256));
    sparc_status st = ensure_red(c, 2 * (size_t)nblk);
    if (st != SPARC_OK) return st;
    k_minmax_part<<<nblk, 256, 0, c->stream>>>(c->veff, c->nd, c->red);
    k_bounds<<<1, 256, 0, c->stream>>>(c->red, nblk, c->kin_bound, c->nl.nl_lo, c->nl.nl_hi, c->scal + S_LO,
                                      c->scal + S_HI);
    SG_CHECK_LAUNCH(c);
    return SPARC_OK;
}

static sparc_status check_block(sparc_gpu_ctx c, int prec, const void* X, int ncol, long ldx, const char* who) {
    if (prec != SPARC_FP64 && prec != SPARC_FP32) return set_err(c, SPARC_ERR_ARG, std::string(who) + ": bad precision");
    if (!X) return set_err(c, SPARC_ERR_ARG, std::string(who) + ": null block");
    if (ncol < 1 || ncol > c->n_states) return set_err(c, SPARC_ERR_ARG, std::string(who) + ": ncol out of range");
    if (ldx < c->nd) return set_err(c, SPARC_ERR_ARG, std::string(who) + ": ldx < N_d");
    return SPARC_OK;
}

static bool overlaps(const void* a, const void* b, size_t bytes) {
    const char* pa = (const char*)a;
    const char* pb = (const char*)b;
    return pa < pb + bytes && pb < pa + bytes;
}

}  // namespace sg

using namespace sg;

extern "C" {

sparc_status sparc_gpu_apply_H(sparc_gpu_ctx c, sparc_prec prec, const void* d_X, void* d_Y, int ncol, long ldx) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    sparc_status st = check_block(c, prec, d_X, ncol, ldx, "apply_H");
    if (st != SPARC_OK) return st;
    if (!d_Y) return set_err(c, SPARC_ERR_ARG, "apply_H: null output");
    size_t es = prec == SPARC_FP64 ? 8 : 4;
    size_t bytes = ((size_t)(ncol - 1) * ldx + c->nd) * es;
    if (overlaps(d_X, d_Y, bytes)) return set_err(c, SPARC_ERR_ARG, "apply_H: X and Y overlap");
    if (prec == SPARC_FP64) return apply_impl<double>(c, (const double*)d_X, (double*)d_Y, ncol, ldx);
    return apply_impl<float>(c, (const float*)d_X, (float*)d_Y, ncol, ldx);
}

sparc_status sparc_gpu_chebyshev_filter(sparc_gpu_ctx c, sparc_prec prec, void* d_X, void* d_work, int ncol,
                                        long ldx, int degree, double a, double b, double a0) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    sparc_status st = check_block(c, prec, d_X, ncol, ldx, "chebyshev_filter");
    if (st != SPARC_OK) return st;
    if (!d_work) return set_err(c, SPARC_ERR_ARG, "chebyshev_filter: null work block");
    if (degree < 1 || degree > 10000) return set_err(c, SPARC_ERR_ARG, "chebyshev_filter: degree out of range");
    if (!(a0 < a && a < b) || !std::isfinite(a0) || !std::isfinite(b))
        return set_err(c, SPARC_ERR_ARG, "chebyshev_filter: need a0 < a < b");
    size_t es = prec == SPARC_FP64 ? 8 : 4;
    size_t bytes = ((size_t)(ncol - 1) * ldx + c->nd) * es;
    if (overlaps(d_X, d_work, bytes)) return set_err(c, SPARC_ERR_ARG, "chebyshev_filter: X and work overlap");
    k_set3<<<1, 1, 0, c->stream>>>(c->scal + S_A, a, b, a0);
    SG_CHECK_LAUNCH(c);
    if (prec == SPARC_FP64) return filter_impl<double>(c, (double*)d_X, (double*)d_work, ncol, ldx, degree);
    return filter_impl<float>(c, (float*)d_X, (float*)d_work, ncol, ldx, degree);
}

}  // extern "C"
