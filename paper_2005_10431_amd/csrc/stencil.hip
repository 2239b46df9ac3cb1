// Matrix-free Hamiltonian and the Chebyshev recurrence built on it.
//
// H x = -1/2 Delta_h x + V_eff x + sum_I sum_lm gamma_Il chi_Ilm (dV chi_Ilm^T x)
// (Sec. 2 eq. (1); matrix-free stencil and outer-product nonlocal term as in
// Sec. 2.1).  The scaled three-term Chebyshev recurrence of the CheFSI filter
// (Sec. 2.1) is fused into the epilogue of the stencil sweep, so one sweep
// streams X_k (stencil operand), X_{k-1} (recurrence term) and writes X_{k+1}
// over X_{k-1}: 3 block-sized streams per filter degree.  With projectors a
// separate pass before each sweep forms the projections D = gamma dV chi^T X_k
// by reading the block once (k_proj_stream), and the sweep adds chi D point
// by point.
//
// Sweep kernel layout (one workgroup = one orbital x one y-slab x all z):
//  - the slab is `ty` full x-rows; periodic x wraps inside LDS (padded rows),
//    so only y needs halo rows, read from L2 where a neighbouring slab of the
//    same orbital (mapped to the same XCD, see the block mapping below)
//    loaded them recently enough, else from the last-level cache or HBM;
//  - z is marched with a register ring of RING = 13 + PR planes per thread:
//    planes z-6 .. z+6 in use and PR planes in flight, so every point of X_k
//    is fetched once per sweep (plus the 12 periodic wrap planes);
//  - the halo rows, X_{k-1}, V_eff and the nonlocal point words of the
//    coming planes sit in PQ-deep register queues, so each load has PQ plane
//    steps to land; the nonlocal pair records are loaded two planes ahead;
//  - two LDS plane buffers alternate so one barrier per plane suffices.
#include <cmath>
#include <map>
#include <mutex>
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
    int grp;          // orbitals whose copies of a slab are dispatched side by side
    // -1/2 Delta_h with the y and z coefficients proportional to the x ones
    // (same weights over h_y^2, h_z^2): ck[q] multiplies
    // (x-pair + ry y-pair + rz z-pair) at distance q, c0 the point itself
    T c0, ck[kMaxHalfOrder + 1], ry, rz;
    const T* veff;
    // nonlocal part (per-slab pair tables, see build_pair_tables)
    const uint64_t* pe8;
    const CandInfo* slab_cand;
    const int* slab_k;
    const SweepPair* pairs;
    const int* pair_off;
    int kmax, xw, pmax;
    const double* atom_pos;  // 3 n_atoms
    T inv_rc2, N0, N1, hx;
    const T* D;       // gamma-scaled projections of x: column j at D + j*ldD, 4 per atom
    int ldD;
    const double* params;  // a, b, a0 on the device
    int step;
    int ncol;
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

constexpr int kRing = 16;            // z-ring slots: planes z-6 .. z+6 and 3 in flight
constexpr int kRingAhead = kRing - 2 * kMaxHalfOrder - 1;
constexpr int kQueue = 2;            // depth of the halo / X_{k-1} / V_eff / point-word queues
constexpr int kSlots = 7;            // pair slots of a point word (byte 0xFF: empty)
constexpr int kPairSlots = 256;      // pair records per plane (index 255: the null pair)
static_assert(kRing % kQueue == 0, "the unrolled step count must cycle every queue");
// Workgroups of the nonlocal sweep are capped at 768 threads (3 waves per
// SIMD) so that the pair tables and the point-word queue fit in registers
// beside the z-ring without spilling.
constexpr int kNlThreads = 768;

// One pair record of a plane in LDS: the pair's contribution at grid x of
// its segment is ex[x] (A'' + B' x), with ex[x] read at byte address
// exb + 8 x (or 4 x in FP32) in LDS.
template <typename T>
struct alignas(2 * sizeof(T) == 16 ? 32 : 16) PairLds {
    T A, B;
    int exb;
};

// LDS of one sweep workgroup, in this order: two padded plane buffers; with
// projectors: the ex tables (K xw, then nx zeros for the null pair), the
// input projections (4 K), delta (K), cxb (K, int), the slab's plane list
// offsets (nz + 1, int), and the pair records of two planes (2 x 256; record
// 255 is the null pair of empty point slots).
struct SweepLds {
    size_t planes, ex, din, delta, cxb, poff, rec, total;
};

__host__ __device__ inline size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

template <typename T>
__host__ __device__ inline SweepLds sweep_lds_layout(int ty, int nx, int nz, int K, int xw, bool nl) {
    SweepLds L{};
    size_t o = 0;
    L.planes = o;
    o += align16(2 * (size_t)(ty + 2 * kMaxHalfOrder) * (nx + 2 * kMaxHalfOrder) * sizeof(T));
    if (nl) {
        L.ex = o;
        o += align16(((size_t)K * xw + nx) * sizeof(T));
        L.din = o;
        o += align16(4 * (size_t)K * sizeof(T));
        L.delta = o;
        o += align16((size_t)K * sizeof(T));
        L.cxb = o;
        o += align16((size_t)K * sizeof(int));
        L.poff = o;
        o += align16(((size_t)nz + 1) * sizeof(int));
        L.rec = o;
        o += align16(2 * (size_t)kPairSlots * sizeof(PairLds<T>));
    }
    L.total = o;
    return L;
}

size_t nl_sweep_lds_bytes(int ty, int nx, int nz, int K, int xw, size_t tsize) {
    return tsize == 8 ? sweep_lds_layout<double>(ty, nx, nz, K, xw, true).total
                      : sweep_lds_layout<float>(ty, nx, nz, K, xw, true).total;
}

int nl_sweep_max_threads() { return kNlThreads; }

template <typename T>
struct SweepShared {
    T* buf0;
    T* buf1;
    // nonlocal tables of the slab
    T* ex;       // ex[k * xw + i] = exp(-(delta_k + i hx)^2 / rc^2); then nx zeros
    T* din;      // din[4 k + lm]: input projections of candidate k's atom
    T* delta;    // x offset of candidate k's first ex entry from its centre (Bohr)
    int* cxb;    // grid x of candidate k's first ex entry
    int* poff;   // poff[z]: start of plane z's pair list in the pair array (z = 0 .. nz)
    PairLds<T>* rec;  // rec[par * 256 + j]: pair j of a plane of parity par
    int exoff;   // byte offset of ex in the workgroup's LDS
};

// Pair record j of plane z's list (n = 0: no pair).
struct PairRec {
    int k, n;
    double eyez, dy, dz;
};

__device__ inline PairRec load_pair(const SweepPair* __restrict__ pairs, const int* poff, int z, int j) {
    PairRec r;
    const int o0 = poff[z], o1 = poff[z + 1];
    r.k = 0;
    r.n = 0;
    r.eyez = r.dy = r.dz = 0.0;
    if (j < o1 - o0) {
        const SweepPair P = pairs[o0 + j];
        r.k = P.k;
        r.n = P.n;
        r.eyez = P.eyez;
        r.dy = P.dy;
        r.dz = P.dz;
    }
    return r;
}

// The record of one plane's pair.  A pair's contribution at grid x of its
// segment is ex(i) (A' + B' i), i = x - cxb_k:
//   chi_s D_s + chi_p . D_p = ex(i) eyez (N0 D_s + N1 (dx D_px + dy D_py + dz D_pz)),
//   dx = delta_k + i hx  =>  A' = eyez (N0 D_s + N1 (dy D_py + dz D_pz + delta_k D_px)),
//                           B' = eyez N1 hx D_px;
// it is stored as A'' = A' - B' cxb_k, so that the contribution is
// ex (A'' + B' x), with the LDS byte offset of the pair's row of the ex
// table shifted by -cxb_k entries, so that x indexes it.
template <typename T>
__device__ inline void pair_record(const SweepArgs<T>& a, const SweepShared<T>& sh, const PairRec& r, int j,
                                   int par) {
    if (r.n == 0) return;
    const int k = r.k;
    const T eyez = (T)r.eyez, dy = (T)r.dy, dz = (T)r.dz;
    const T fs = eyez * a.N0, fx = eyez * a.N1;
    const T* D = sh.din + 4 * k;
    const T A = fs * D[0] + fx * (dy * D[2] + dz * D[3] + sh.delta[k] * D[1]);
    const T B = fx * a.hx * D[1];
    const int c0 = sh.cxb[k];
    PairLds<T>& R = sh.rec[par * kPairSlots + j];
    R.A = A - B * (T)c0;
    R.B = B;
    R.exb = sh.exoff + (k * a.xw - c0) * (int)sizeof(T);
}

// The sweep.  MODE: 0 out = H x; 1 first filter step; 2 filter step `step`
// (>= 2) with xprev = X_{k-1} (may alias out).  NL: projectors present (the
// projections of x are in a.D).  HM: halo values per thread and plane.
//
// One z-plane step at ring phase U (z = z0 + U).  On entry the LDS buffer of
// parity U holds plane z (own rows with x-wrap padding and halo rows) and the
// pair records of plane z, written during the previous step.
//  1. barrier, then the nonlocal term of plane z from the pair records (right
//     after the barrier, where the fewest values are live);
//  2. issue the loads of the halo values of plane z + PQ, of ring plane
//     z + 6 + PR (plane indices wrap, so the loads are unconditional) and of
//     the pair records of plane z + 2;
//  3. stencil + potential + recurrence for plane z, store;
//  4. load X_{k-1}, V_eff and the point word of plane z + PQ into the queue
//     slot plane z has freed;
//  5. pair records of plane z + 1 (loaded during the previous step) into the
//     other record buffer; plane z + 1 into the other LDS buffer.
// The nonlocal term takes NSL slots of the point word without a branch (empty
// slots name the null pair, whose ex entries are zero), or with NSL = 4 four
// slots and the other three in a branch; a loop inside the unrolled step
// would keep every value live across it.  Threads without a point of the slab
// (ragged slab, padding to 64) load valid clamped addresses and compute on
// them, but never store.
template <typename T, bool NL, int MODE, int HM, int NSL = 4>
__global__ __launch_bounds__(NL ? kNlThreads : 1024) void k_hsweep(SweepArgs<T> a) {
    constexpr int NO = kMaxHalfOrder;
    constexpr int RING = kRing, PR = kRingAhead, PQ = kQueue;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int W = nx + 2 * NO;
    const int R = a.ty + 2 * NO;

    // Hardware dispatches block b to XCD b % 8.  Give each XCD a contiguous
    // range of logical tiles so that the y-slabs of one orbital (which read
    // each other's rows as halos) share an L2.  Within a group of grp
    // orbitals the logical order is slab-major, so that the grp copies of a
    // slab (which read the same V_eff rows and point words) run side by side.
    const int nblk = gridDim.x, bid = blockIdx.x;
    const int qn = nblk / 8, rn = nblk % 8;
    const int xcd = bid % 8, bslot = bid / 8;
    const int logical = xcd * qn + min(xcd, rn) + bslot;
    const int gsz = a.grp * a.ntiles_y;
    const int gi = logical / gsz, gr = logical - gi * gsz;
    const int gcols = min(a.grp, a.ncol - gi * a.grp);   // the last group may be short
    const int tile = gr / gcols;
    const int col = gi * a.grp + (gr - tile * gcols);
    const int y0 = tile * a.ty;
    const int tyn = min(a.ty, ny - y0);

    const int t = threadIdx.x;
    const int nt = blockDim.x;
    const int lx = t % nx, ly = t / nx;
    const bool active = ly < tyn;
    const long plane = (long)nx * ny;

    SweepShared<T> sh;
    {
        const SweepLds L = sweep_lds_layout<T>(a.ty, nx, nz, NL ? a.kmax : 0, a.xw, NL);
        sh.buf0 = reinterpret_cast<T*>(smem_raw + L.planes);
        sh.buf1 = sh.buf0 + R * W;
        sh.ex = reinterpret_cast<T*>(smem_raw + L.ex);
        sh.din = reinterpret_cast<T*>(smem_raw + L.din);
        sh.delta = reinterpret_cast<T*>(smem_raw + L.delta);
        sh.cxb = reinterpret_cast<int*>(smem_raw + L.cxb);
        sh.poff = reinterpret_cast<int*>(smem_raw + L.poff);
        sh.rec = reinterpret_cast<PairLds<T>*>(smem_raw + L.rec);
        sh.exoff = (int)L.ex;
    }
    if (NL) {
        const int K = a.slab_k[tile];
        const CandInfo* ci = a.slab_cand + (long)tile * a.kmax;
        const T* Dc = a.D + (long)col * a.ldD;
        for (int k = t; k < K; k += nt) {
            const CandInfo c = ci[k];
            sh.delta[k] = (T)((double)c.ixlo * (double)a.hx - a.atom_pos[3 * c.atom]);
            sh.cxb[k] = c.ixlo - c.sx * nx;
            for (int lm = 0; lm < 4; ++lm) sh.din[4 * k + lm] = Dc[4 * c.atom + lm];
        }
        for (int j = t; j < K * a.xw + nx; j += nt) {
            T v = 0;
            if (j < K * a.xw) {
                const int k = j / a.xw, i = j - k * a.xw;
                const T dx = (T)(ci[k].ixlo + i) * a.hx - (T)a.atom_pos[3 * ci[k].atom];
                v = exp(-dx * dx * a.inv_rc2);
            }
            sh.ex[j] = v;
        }
        for (int z = t; z <= nz; z += nt) sh.poff[z] = a.pair_off[tile * nz + z];
        // the null pair of both plane parities: ex = 0 over the whole row
        if (t < 2) {
            PairLds<T>& N = sh.rec[t * kPairSlots + 255];
            N.A = 0;
            N.B = 0;
            N.exb = sh.exoff + K * a.xw * (int)sizeof(T);
        }
        __syncthreads();
        // pair records of plane 0
        for (int j = t; j < a.pmax; j += nt) pair_record<T>(a, sh, load_pair(a.pairs, sh.poff, 0, j), j, 0);
    }
    // pair records in flight: rec[p] holds the record of the next plane of
    // parity p (plane 1 to start with; plane 2 is loaded by the first step)
    PairRec rec[2];
    rec[0].k = rec[0].n = 0;
    rec[0].eyez = rec[0].dy = rec[0].dz = 0.0;
    if (NL && t < a.pmax) {
        rec[1] = load_pair(a.pairs, sh.poff, 1 < nz ? 1 : 0, t);
    } else {
        rec[1] = rec[0];
    }

    const T* __restrict__ xc = a.x + (long)col * a.ldx;
    T* __restrict__ oc = a.out + (long)col * a.ldx;
    const T* __restrict__ pc = a.xprev ? a.xprev + (long)col * a.ldx : xc;
    const long pxy = lx + (long)nx * (y0 + (active ? ly : 0));
    const int lrow = ((active ? ly : 0) + NO) * W + NO + lx;
    // halo rows: 2 NO rows of nx values per plane, spread over the threads
    int goff[HM], loff[HM], poff[HM];
    int hn = 0;
    const int nhalo = 2 * NO * nx;
#pragma unroll
    for (int i = 0; i < HM; ++i) {
        const int e = t + i * nt;
        goff[i] = 0;
        loff[i] = 0;
        poff[i] = -1;
        if (e < nhalo) {
            hn = i + 1;
            int hr = e / nx, hx = e - hr * nx;
            int lr, gy;
            if (hr < NO) {
                lr = hr;
                gy = y0 - NO + hr;
            } else {
                lr = NO + tyn + (hr - NO);
                gy = y0 + tyn + (hr - NO);
            }
            gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
            goff[i] = hx + nx * gy;
            loff[i] = lr * W + NO + hx;
            if (hx < NO) poff[i] = loff[i] + nx;
            if (hx >= nx - NO) poff[i] = loff[i] - nx;
        }
    }

    double alpha_d, c_d, beta_d;
    filter_coefs(a.params, MODE, a.step, alpha_d, c_d, beta_d);
    const T alpha = (T)alpha_d, cshift = (T)c_d, beta = (T)beta_d;
    auto wz = [nz](int z) { return z >= nz ? z - nz : (z < 0 ? z + nz : z); };
    const T lxd = (T)lx;
    const int lxb = lx * (int)sizeof(T);

    T q[RING];
    T hq[PQ][HM];
    T xp[PQ], ve[PQ];
    uint64_t w8[PQ];
    // ring: planes -6 .. 5 + PR (slot = plane mod RING); queues: planes 0 .. PQ-1
#pragma unroll
    for (int j = -NO; j <= NO - 1 + PR; ++j) q[(j + 2 * RING) % RING] = xc[pxy + (long)wz(j) * plane];
#pragma unroll
    for (int j = 0; j < PQ; ++j) {
        const long zo = (long)wz(j) * plane;
        xp[j] = MODE == 2 ? __builtin_nontemporal_load(&pc[pxy + zo]) : (T)0;
        ve[j] = a.veff[pxy + zo];
        w8[j] = NL ? a.pe8[pxy + zo] : ~0ull;
    }
#pragma unroll
    for (int j = 1; j < PQ; ++j)
#pragma unroll
        for (int i = 0; i < HM; ++i) hq[j][i] = (i < hn) ? xc[goff[i] + (long)wz(j) * plane] : (T)0;
    // plane 0 into LDS buffer 0
    if (active) {
        sh.buf0[lrow] = q[0];
        if (lx < NO) sh.buf0[lrow + nx] = q[0];
        if (lx >= nx - NO) sh.buf0[lrow - nx] = q[0];
    }
#pragma unroll
    for (int i = 0; i < HM; ++i)
        if (i < hn) {
            const T v = xc[goff[i]];
            sh.buf0[loff[i]] = v;
            if (poff[i] >= 0) sh.buf0[poff[i]] = v;
        }

    for (int z0 = 0; z0 < nz; z0 += RING) {
#pragma unroll
        for (int U = 0; U < RING; ++U) {
            const int z = z0 + U;
            if (z >= nz) break;
            const int P = U & 1, PN = (U + 1) & 1, QS = U % PQ, QN = (U + 1) % PQ;
            __syncthreads();
            // nonlocal term of plane z: the sum over the pairs whose
            // segment holds this point of chi_s D_s + chi_p . D_p =
            // ex (A'' + B' x)
            T nl = 0;
            if (NL) {
                const uint64_t w = active ? w8[QS] : ~0ull;
                const PairLds<T>* rb = sh.rec + P * kPairSlots;
                auto slot = [&](int sl) {
                    const PairLds<T>& R8 = rb[(int)((w >> (8 * sl)) & 0xFFull)];
                    const T e = *reinterpret_cast<const T*>(smem_raw + (R8.exb + lxb));
                    nl += e * (R8.A + R8.B * lxd);
                };
                if constexpr (NSL == 4) {
                    // four slots for every point; the other three only where
                    // a point of the wave lies in more than four supports
                    // (about one point in a hundred)
#pragma unroll
                    for (int sl = 0; sl < 4; ++sl) slot(sl);
                    if (((uint32_t)(w >> 32) | 0xFF000000u) != 0xFFFFFFFFu) {
#pragma unroll
                        for (int sl = 4; sl < kSlots; ++sl) slot(sl);
                    }
                } else {
                    // NSL slots for every point, no branch (the tables hold
                    // at most NSL pairs per point)
#pragma unroll
                    for (int sl = 0; sl < NSL; ++sl) slot(sl);
                }
            }
            // 2. loads of later planes
            {
                const long zo = (long)wz(z + PQ) * plane;
#pragma unroll
                for (int i = 0; i < HM; ++i) hq[QS][i] = (i < hn) ? xc[goff[i] + zo] : (T)0;
                q[(U + NO + PR + RING) % RING] = xc[pxy + (long)wz(z + NO + PR) * plane];
            }
            // the record of plane z + 2, two steps ahead of its use
            if (NL && t < a.pmax) rec[P] = load_pair(a.pairs, sh.poff, z + 2 < nz ? z + 2 : 0, t);
            // 3. plane z
            const T* rp = (P ? sh.buf1 : sh.buf0) + lrow;
            const int C = U % RING;
            T lap = a.c0 * q[C];
#pragma unroll
            for (int k = 1; k <= NO; ++k) {
                T s = (rp[k] + rp[-k]) + a.ry * (rp[k * W] + rp[-k * W]);
                s += a.rz * (q[(U + k) % RING] + q[(U + RING - k) % RING]);
                lap += a.ck[k] * s;
            }
            T hv = lap + ve[QS] * q[C] + nl;
            T o;
            if (MODE == 0) {
                o = hv;
            } else {
                o = alpha * (hv - cshift * q[C]);
                if (MODE == 2) o += beta * xp[QS];
            }
            if (active) __builtin_nontemporal_store(o, &oc[pxy + (long)z * plane]);
            // 4. queue loads of plane z + PQ
            {
                const long zo = (long)wz(z + PQ) * plane;
                if (MODE == 2) xp[QS] = __builtin_nontemporal_load(&pc[pxy + zo]);
                ve[QS] = a.veff[pxy + zo];
                if (NL) w8[QS] = a.pe8[pxy + zo];
            }
            // 5. pair records and LDS plane of z + 1
            if (NL && z + 1 < nz && t < a.pmax) pair_record<T>(a, sh, rec[PN], t, PN);
            T* nbuf = P ? sh.buf0 : sh.buf1;
            const int CN = (U + 1) % RING;
            if (active) {
                nbuf[lrow] = q[CN];
                if (lx < NO) nbuf[lrow + nx] = q[CN];
                if (lx >= nx - NO) nbuf[lrow - nx] = q[CN];
            }
#pragma unroll
            for (int i = 0; i < HM; ++i)
                if (i < hn) {
                    nbuf[loff[i]] = hq[QN][i];
                    if (poff[i] >= 0) nbuf[poff[i]] = hq[QN][i];
                }
        }
    }
}

// Projections by streaming the block once.  D(4a+lm, j) = gamma_lm dV
// sum_p chi_lm(p) X(p, j) over the image points of atom a's support.  A
// workgroup takes one y-slab of the nonlocal sweep (the same slabs and pair
// tables), a range of z-planes and NW orbitals, one per wave; the waves
// share the slab's ex tables and otherwise run independently (no workgroup
// barrier after set-up).  A wave copies each plane of its orbital's slab
// into its own LDS (coalesced rows, two planes in flight ahead) and, 64
// pairs (candidate k, row, segment) at a time, one per lane, forms
//   S0 = sum_i ex_k(i) X(i),  S1 = sum_i i ex_k(i) X(i)   (i: ex index),
// whose contributions to candidate k are, with f_s = eyez N0, f_p = eyez N1,
//   s: f_s S0,  p_x: f_p (delta_k S0 + hx S1),  p_y: f_p dy S0,  p_z: f_p dz S0.
// The lane of the first pair of each candidate's run (never split over two
// groups of 64) adds the run's contributions, in row order, to the
// candidate's accumulators; planes are taken in order.  Every sum is in
// double and in a fixed order, so the result is bitwise reproducible.  The
// accumulators of the (z range, slab, candidate) are written as partials,
// which k_proj_reduce sums per atom.
constexpr int kProjWaveVals = 12;   // plane values per lane: ty nx <= 768

struct ProjLds {
    size_t ex, delta, poff, wave, wave_bytes, total;
};

__host__ __device__ inline ProjLds proj_lds_layout(int ty, int nx, int nz, int K, int xw, int NW, size_t ts) {
    ProjLds L{};
    size_t o = 0;
    L.ex = o;
    o += align16((size_t)K * xw * ts);
    L.delta = o;
    o += align16((size_t)K * sizeof(double));
    L.poff = o;
    o += align16(((size_t)nz + 1) * sizeof(int));
    // per wave: its plane (64 x kProjWaveVals values, of which ty nx are
    // used), 64 x 4 pair contributions, K x 4 FP64 accumulators (the ex
    // table, the plane and the contributions in the block's precision)
    L.wave_bytes = align16((size_t)64 * kProjWaveVals * ts) + align16(64 * 4 * ts) +
                   align16((size_t)K * 4 * sizeof(double));
    L.wave = o;
    o += (size_t)NW * L.wave_bytes;
    L.total = o;
    return L;
}

size_t nl_proj_lds_bytes(int ty, int nx, int nz, int K, int xw, int NW, size_t tsize) {
    return proj_lds_layout(ty, nx, nz, K, xw, NW, tsize).total;
}

struct ProjArgs {
    long ldx;
    int nx, ny, nz, ty, ntiles_y, ncol, nw;
    int zsplit, zlen;          // z ranges per slab and planes per range
    const CandInfo* slab_cand;
    const int* slab_k;
    const ProjPair* ppairs;
    const int* pair_off;
    int kmax, xw;
    const double* atom_pos;
    double inv_rc2, N0, N1, hx;
    double cq;                 // exp(-2 hx^2 / rc^2)
    double* part;              // [((zr * ntiles_y + slab) * kmax + k) * ncol + col] * 4
};

// LDS writes of one lane made visible to the other lanes of its wave
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__global__ __launch_bounds__(512) void k_proj_stream(const T* __restrict__ x, ProjArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int nx = a.nx, ny = a.ny;
    const long plane = (long)nx * ny;
    const int NW = a.nw;
    const int nchunk = (a.ncol + NW - 1) / NW;
    // block -> (column chunk, z range, slab), slabs fastest
    int bid = blockIdx.x;
    const int tile = bid % a.ntiles_y;
    bid /= a.ntiles_y;
    const int zr = bid % a.zsplit;
    const int chunk = bid / a.zsplit;
    if (chunk >= nchunk) return;
    const int y0 = tile * a.ty, tyn = min(a.ty, ny - y0);
    const int zb = zr * a.zlen, ze = min(a.nz, zb + a.zlen);
    const int t = threadIdx.x, nt = blockDim.x;
    const int K = a.slab_k[tile];
    const CandInfo* ci = a.slab_cand + (long)tile * a.kmax;
    const int* poffg = a.pair_off + (long)tile * a.nz;

    const ProjLds L = proj_lds_layout(a.ty, nx, a.nz, a.kmax, a.xw, NW, sizeof(T));
    T* ex = reinterpret_cast<T*>(smem_raw + L.ex);
    double* delta = reinterpret_cast<double*>(smem_raw + L.delta);
    int* poff = reinterpret_cast<int*>(smem_raw + L.poff);   // plane lists of z in [zb, ze]
    for (int j = t; j < K * a.xw; j += nt) {
        const int k = j / a.xw, i = j - k * a.xw;
        const double dx = (double)(ci[k].ixlo + i) * a.hx - a.atom_pos[3 * ci[k].atom];
        ex[j] = (T)exp(-dx * dx * a.inv_rc2);
    }
    for (int k = t; k < K; k += nt) delta[k] = (double)ci[k].ixlo * a.hx - a.atom_pos[3 * ci[k].atom];
    for (int z = zb + t; z <= ze; z += nt) poff[z - zb] = poffg[z];
    __syncthreads();

    const int w = t >> 6, lane = t & 63;
    const int col = chunk * NW + w;
    if (col >= a.ncol) return;
    unsigned char* wb = smem_raw + L.wave + (size_t)w * L.wave_bytes;
    T* buf = reinterpret_cast<T*>(wb);
    T* psum = reinterpret_cast<T*>(wb + align16((size_t)64 * kProjWaveVals * sizeof(T)));
    double* acc = reinterpret_cast<double*>(reinterpret_cast<unsigned char*>(psum) + align16(64 * 4 * sizeof(T)));
    for (int j = lane; j < K * 4; j += 64) acc[j] = 0.0;

    // The slab's rows of one plane are contiguous: value e of the plane is
    // global offset base + e and LDS offset e.  Loads and stores take no
    // branch (values past the plane and planes past the range read clamped
    // valid addresses and land in unused LDS), so that the loads of later
    // planes stay in flight while a plane is processed.
    const int nvals = tyn * nx;
    const T* xs = x + (long)col * a.ldx + (long)nx * y0;
    long eoff[kProjWaveVals];
#pragma unroll
    for (int i = 0; i < kProjWaveVals; ++i) eoff[i] = min(lane + 64 * i, nvals - 1);
    T va[kProjWaveVals], vb[kProjWaveVals];
    auto load_plane = [&](T* v, int z) {
        const long zo = (long)min(z, ze - 1) * plane;
#pragma unroll
        for (int i = 0; i < kProjWaveVals; ++i) v[i] = xs[zo + eoff[i]];
    };
    auto store_plane = [&](const T* v) {
#pragma unroll
        for (int i = 0; i < kProjWaveVals; ++i) buf[lane + 64 * i] = v[i];
    };
    // The pairs of a plane, 64 per group (lane = pair); the first three
    // groups are loaded a plane ahead.  Lanes past the list load a clamped
    // valid record and ignore it (the record is not touched before use, so
    // that its load stays in flight).
    constexpr int kGroups = 3;
    auto load_recs = [&](ProjPair* R, int z) {
        const int zc = min(z, ze - 1) - zb;
        const int o0 = poff[zc], np = poff[zc + 1] - o0;
#pragma unroll
        for (int g = 0; g < kGroups; ++g) {
            const int j = 64 * g + lane;
            R[g] = a.ppairs[max(0, o0 + min(j, np - 1))];
        }
    };
    auto do_group = [&](const ProjPair& Q, bool ok) {
        const int k = Q.kw & 1023, xo = (Q.kw >> 10) & 255, run = Q.kw >> 18;
        const int row = Q.rw & 255, xlo = (Q.rw >> 8) & 255, n = ok ? (int)(Q.rw >> 16) : 0;
        double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0;
        if (n > 0) {
            // a segment's arithmetic runs in the block's precision (the
            // per-atom sums below stay in FP64)
            using R = T;
            const T* xr = buf + row * nx + xlo;
            const T* er = ex + k * a.xw + xo;
            // The Gaussian along the segment by its recurrence: with
            // ex(i) = exp(-(delta + i hx)^2 / rc^2) and g(i) = ex(i+1)/ex(i),
            // g(i+1) = g(i) exp(-2 hx^2 / rc^2); two multiplies per point in
            // place of an LDS read (ex >= exp(-rcut^2/rc^2) > 0 on a support).
            R ev = (R)er[0];
            R gq = n > 1 ? (R)(er[1] / er[0]) : (R)0;
            const R cq = (R)a.cq;
            auto next = [&](R x) {
                const R v = ev * x;
                ev *= gq;
                gq *= cq;
                return v;
            };
            // four points at a time: with e_u = ex(i+u) X(i+u),
            //   S0 += sum_u e_u,  S1 += (xo+i) sum_u e_u + (e_1 + 2 e_2 + 3 e_3)
            R s0 = 0, s1 = 0, ii = (R)xo;
            int i = 0;
            for (; i + 4 <= n; i += 4) {
                const R e0 = next(xr[i]), e1 = next(xr[i + 1]), e2 = next(xr[i + 2]), e3 = next(xr[i + 3]);
                const R sum = (e0 + e1) + (e2 + e3);
                s0 += sum;
                s1 += ii * sum + fma((R)3, e3, fma((R)2, e2, e1));
                ii += (R)4;
            }
            if (i < n) {
                // the last one to three points
                const R e0 = next(xr[i]);
                const R e1 = i + 1 < n ? next(xr[i + 1]) : (R)0;
                const R e2 = i + 2 < n ? next(xr[i + 2]) : (R)0;
                const R sum = (e0 + e1) + e2;
                s0 += sum;
                s1 += ii * sum + fma((R)2, e2, e1);
            }
            const double fs = Q.eyez * a.N0, fp = Q.eyez * a.N1;
            c0 = fs * s0;
            c1 = fp * (delta[k] * s0 + a.hx * s1);
            c2 = fp * Q.dy * s0;
            c3 = fp * Q.dz * s0;
        }
        T* ps = psum + lane * 4;
        ps[0] = c0;
        ps[1] = c1;
        ps[2] = c2;
        ps[3] = c3;
        wave_sync();
        if (n > 0 && run > 0) {
            double* ac = acc + k * 4;
            double d0 = ac[0], d1 = ac[1], d2 = ac[2], d3 = ac[3];
            for (int r = 0; r < run; ++r) {
                const T* q = psum + (lane + r) * 4;
                d0 += q[0];
                d1 += q[1];
                d2 += q[2];
                d3 += q[3];
            }
            ac[0] = d0;
            ac[1] = d1;
            ac[2] = d2;
            ac[3] = d3;
        }
        wave_sync();
    };
    auto do_plane = [&](const ProjPair* R, int z) {
        const int o0 = poff[z - zb], np = poff[z - zb + 1] - o0;
        if (np > 0) do_group(R[0], lane < np);
        if (np > 64) do_group(R[1], 64 + lane < np);
        if (np > 128) do_group(R[2], 128 + lane < np);
        for (int g = kGroups; 64 * g < np; ++g) {
            const int j = 64 * g + lane;
            do_group(a.ppairs[o0 + min(j, np - 1)], j < np);
        }
    };
    ProjPair ra[kGroups], rb[kGroups];
    load_plane(va, zb);
    load_plane(vb, zb + 1);
    load_recs(ra, zb);
    load_recs(rb, zb + 1);
    for (int z = zb; z < ze; z += 2) {
        store_plane(va);
        load_plane(va, z + 2);
        wave_sync();
        do_plane(ra, z);
        load_recs(ra, z + 2);
        if (z + 1 >= ze) break;
        store_plane(vb);
        load_plane(vb, z + 3);
        wave_sync();
        do_plane(rb, z + 1);
        load_recs(rb, z + 3);
    }
    const long row0 = ((long)zr * a.ntiles_y + tile) * a.kmax;
    for (int j = lane; j < K * 4; j += 64) {
        const int k = j >> 2, lm = j & 3;
        a.part[((row0 + k) * a.ncol + col) * 4 + lm] = acc[j];
    }
}

// D(4a+lm, col) = gamma_lm dV sum of atom a's partials: its (slab,
// candidate) entries in table order, and within each the z ranges in order.
template <typename T>
__global__ __launch_bounds__(256) void k_proj_reduce(const double* __restrict__ part, int ncol, int zsplit,
                                                     long zstride, const int* __restrict__ red_off,
                                                     const int* __restrict__ red_idx,
                                                     const double* __restrict__ g4, double dV, T* __restrict__ D,
                                                     int ldD) {
    const int a = blockIdx.x;
    const long q = (long)blockIdx.y * blockDim.x + threadIdx.x;
    if (q >= 4L * ncol) return;
    const int col = (int)(q / 4), lm = (int)(q % 4);
    double s = 0.0;
    for (int e = red_off[a]; e < red_off[a + 1]; ++e)
        for (int zr = 0; zr < zsplit; ++zr) s += part[(zr * zstride + red_idx[e]) * ncol * 4 + q];
    D[(long)col * ldD + 4 * a + lm] = (T)(g4[4 * a + lm] * dV * s);
}

int choose_sweep_ty(int nx, int ny, int max_threads) {
    // tuning override: rows per y-slab
    if (const char* e = std::getenv("SPARC_GPU_SWEEP_TY")) {
        int v = std::atoi(e);
        if (v >= 1 && v <= ny && ((v * nx + 63) / 64) * 64 <= max_threads) return v;
    }
    int maxty = std::max(1, std::min(16, max_threads / nx));
    maxty = std::min(maxty, ny);
    // the largest divisor of ny not above maxty, unless it is small
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

// Slab height of the local sweep: the largest divisor of n_y with at most
// 1024 threads in FP64 and 512 in FP32 (whose lighter threads prefer more
// workgroups per CU), measured best on MI355X at 72 and 120 points per row.
static int local_ty(sparc_gpu_ctx c, size_t tsize) {
    return choose_sweep_ty(c->nx, c->ny, tsize == 8 ? 1024 : 512);
}

template <typename T>
sparc_status launch_hsweep(sparc_gpu_ctx c, const T* x, T* out, const T* xprev, int ncol, long ldx, int mode,
                           int step) {
    hipStream_t stream = c->stream;
    SweepArgs<T> a;
    a.x = x;
    a.out = out;
    a.xprev = xprev;
    a.ldx = ldx;
    a.nx = c->nx;
    a.ny = c->ny;
    a.nz = c->nz;
    const bool nl = !c->sweep_local_only && c->nl_lmax >= 1 && c->nl.n_pe > 0;
    // the FP32 sweep's own slab tables where it has them
    const NonlocalTables& NT = (sizeof(T) == 4 && c->nl32.slab_ty > 0) ? c->nl32 : c->nl;
    a.ty = nl ? NT.slab_ty : local_ty(c, sizeof(T));
    a.ntiles_y = div_up(c->ny, a.ty);
    a.grp = std::max(1, std::min(c->sweep_group, ncol));
    {
        const StencilCoef<T>& cf = coef<T>(c);
        a.c0 = cf.c0;
        for (int k = 0; k <= kMaxHalfOrder; ++k) a.ck[k] = cf.cx[k];
        a.ry = (T)((c->hx * c->hx) / (c->hy * c->hy));
        a.rz = (T)((c->hx * c->hx) / (c->hz * c->hz));
    }
    a.veff = veff_of<T>(c);
    a.pe8 = NT.pe8;
    a.slab_cand = NT.slab_cand;
    a.slab_k = NT.slab_k;
    a.pairs = NT.pairs;
    a.pair_off = NT.pair_off;
    a.kmax = NT.slab_kmax;
    a.xw = NT.slab_xw;
    a.pmax = NT.pair_max;
    a.atom_pos = c->atom_pos;
    {
        const double pi = 3.14159265358979323846;
        const double rc = c->rc_nl > 0 ? c->rc_nl : 1.0;
        const double N0 = std::pow(2.0 / (pi * rc * rc), 0.75);
        a.inv_rc2 = (T)(1.0 / (rc * rc));
        a.N0 = (T)N0;
        a.N1 = (T)((2.0 / rc) * N0);
        a.hx = (T)c->hx;
    }
    a.D = D_of<T>(c);
    a.ldD = 4 * c->n_atoms;
    a.params = c->scal + S_A;
    a.step = step;
    a.ncol = ncol;
    int threads = div_up((long)c->nx * a.ty, 64) * 64;
    if (nl) threads = std::max(threads, div_up(a.pmax, 64) * 64);
    const size_t shmem = sweep_lds_layout<T>(a.ty, c->nx, c->nz, nl ? a.kmax : 0, a.xw, nl).total;
    if (shmem > 160 * 1024) return set_err(c, SPARC_ERR_ARG, "sweep workgroup needs more than 160 KB of LDS");
    if (threads > (nl ? kNlThreads : 1024)) return set_err(c, SPARC_ERR_ARG, "grid x-extent too large for the sweep kernel");
    const long nblocks = (long)ncol * a.ntiles_y;
    if (nblocks > 0x7fffffffL) return set_err(c, SPARC_ERR_ARG, "too many blocks");
    const int hm = div_up(2L * kMaxHalfOrder * c->nx, threads);
    if (hm > 6) return set_err(c, SPARC_ERR_ARG, "grid x-extent too large for the sweep kernel");
    if (nblocks == 0) return SPARC_OK;
    const int slot = prof_begin(c, mode == 2 ? PK_SWEEP : (mode == 1 ? PK_SWEEP1 : PK_APPLY), stream);
    const dim3 g((unsigned)nblocks), b(threads);
    // Nonlocal slots per point: FP64 takes them all without a branch (6 when
    // no point of the tables lies in more than 6 supports, else 7); FP32,
    // whose 4-row slabs need 128 VGPRs or fewer for two workgroups per CU,
    // takes 4 and the rest in a branch.  Measured at 120^3 FP64: 18.3 (6),
    // 18.7 (7) against 18.8 ms (4 + branch); FP32: 12.7 (4 + branch)
    // against 19.6 ms (7).
    const int nsl = sizeof(T) == 8 ? (NT.max_entries <= 6 && c->nl_slots != 7 ? 6 : 7) : 4;
#define SG_LAUNCH_SWEEP(NLV, MV, HMV, NSV) k_hsweep<T, NLV, MV, HMV, NSV><<<g, b, shmem, stream>>>(a)
#define SG_SWEEP_HM(NLV, MV, NSV)                          \
    do {                                                   \
        switch (hm) {                                      \
            case 1: SG_LAUNCH_SWEEP(NLV, MV, 1, NSV); break; \
            case 2: SG_LAUNCH_SWEEP(NLV, MV, 2, NSV); break; \
            case 3: SG_LAUNCH_SWEEP(NLV, MV, 3, NSV); break; \
            case 4: SG_LAUNCH_SWEEP(NLV, MV, 4, NSV); break; \
            case 5: SG_LAUNCH_SWEEP(NLV, MV, 5, NSV); break; \
            default: SG_LAUNCH_SWEEP(NLV, MV, 6, NSV); break; \
        }                                                  \
    } while (0)
#define SG_SWEEP_NL(MV)                                          \
    do {                                                         \
        if constexpr (sizeof(T) == 8) {                          \
            if (nsl == 6) SG_SWEEP_HM(true, MV, 6);              \
            else SG_SWEEP_HM(true, MV, 7);                       \
        } else {                                                 \
            SG_SWEEP_HM(true, MV, 4);                            \
        }                                                        \
    } while (0)
    if (nl) {
        if (mode == 0) SG_SWEEP_NL(0);
        else if (mode == 1) SG_SWEEP_NL(1);
        else SG_SWEEP_NL(2);
    } else {
        if (mode == 0) SG_SWEEP_HM(false, 0, 4);
        else if (mode == 1) SG_SWEEP_HM(false, 1, 4);
        else SG_SWEEP_HM(false, 2, 4);
    }
#undef SG_SWEEP_NL
#undef SG_SWEEP_HM
#undef SG_LAUNCH_SWEEP
    SG_CHECK_LAUNCH(c);
    prof_end(c, slot, stream);
    return SPARC_OK;
}

// Orbitals (waves) per projection workgroup: the most of 8, 4, 2 whose
// LDS fits (SPARC_GPU_PROJ_NB caps it).
static int proj_nw(sparc_gpu_ctx c, size_t tsize) {
    const NonlocalTables& NT = c->nl;
    int nw = (c->proj_nb == 2 || c->proj_nb == 4) ? c->proj_nb : 8;
    while (nw > 1 && nl_proj_lds_bytes(c->nl_ty, c->nx, c->nz, NT.slab_kmax, NT.slab_xw, nw, tsize) > 160 * 1024)
        nw /= 2;
    return nw;
}

template <typename T>
sparc_status launch_projection(sparc_gpu_ctx c, const T* x, int ncol, long ldx, double* part, size_t part_elems) {
    if (c->nl_lmax < 1 || c->nl.n_pe == 0 || ncol == 0) return SPARC_OK;
    hipStream_t stream = c->stream;
    const NonlocalTables& NT = c->nl;
    ProjArgs a;
    a.ldx = ldx;
    a.nx = c->nx;
    a.ny = c->ny;
    a.nz = c->nz;
    a.ty = c->nl_ty;
    a.ntiles_y = div_up(c->ny, a.ty);
    a.slab_cand = NT.slab_cand;
    a.slab_k = NT.slab_k;
    a.ppairs = NT.ppairs;
    a.pair_off = NT.pair_off;
    a.kmax = NT.slab_kmax;
    a.xw = NT.slab_xw;
    a.atom_pos = c->atom_pos;
    {
        const double pi = 3.14159265358979323846;
        const double rc = c->rc_nl;
        const double N0 = std::pow(2.0 / (pi * rc * rc), 0.75);
        a.inv_rc2 = 1.0 / (rc * rc);
        a.N0 = N0;
        a.N1 = (2.0 / rc) * N0;
        a.hx = c->hx;
        a.cq = std::exp(-2.0 * c->hx * c->hx / (rc * rc));
    }
    a.nw = proj_nw(c, sizeof(T));
    const size_t shmem = nl_proj_lds_bytes(a.ty, a.nx, a.nz, a.kmax, a.xw, a.nw, sizeof(T));
    if (shmem > 160 * 1024) return set_err(c, SPARC_ERR_ARG, "projection workgroup needs more than 160 KB of LDS");
    if ((long)a.ty * a.nx > 64L * kProjWaveVals)
        return set_err(c, SPARC_ERR_ARG, "slab too large for the projection kernel");
    // z ranges per slab, from the whole block: enough waves for 32 per
    // compute unit, each range at least 8 planes (the ranges fix the order of
    // the sums, so a block gives the same result however its columns are
    // launched)
    const long base = (long)a.ntiles_y * div_up(ncol, a.nw);
    a.zsplit = (int)std::max(1L, std::min((long)std::max(1, a.nz / 8), (long)div_up(8192L, base * a.nw)));
    a.zlen = div_up(a.nz, a.zsplit);
    a.zsplit = div_up(a.nz, a.zlen);
    const size_t per_col = (size_t)a.zsplit * a.ntiles_y * a.kmax * 4;
    int chunk = ncol;
    if (part) {
        // caller memory: as many columns at a time as it holds
        if (per_col > part_elems)
            return set_err(c, SPARC_ERR_ARG, "projection partials of one column exceed the fixed scratch array");
        chunk = (int)std::min<size_t>((size_t)ncol, part_elems / per_col);
    } else {
        const size_t need = per_col * ncol;
        if (c->nl_part_elems < need) {
            if (c->nl_part) {
                SG_HIP(c, hipStreamSynchronize(stream));
                SG_HIP(c, hipFree(c->nl_part));
                c->nl_part = nullptr;
                c->nl_part_elems = 0;
            }
            SG_HIP(c, hipMalloc((void**)&c->nl_part, need * sizeof(double)));
            c->nl_part_elems = need;
        }
        part = c->nl_part;
    }
    a.part = part;
    const int slot = prof_begin(c, PK_PROJ, stream);
    for (int c0 = 0; c0 < ncol; c0 += chunk) {
        a.ncol = std::min(chunk, ncol - c0);
        const long nblocks = (long)a.ntiles_y * div_up(a.ncol, a.nw) * a.zsplit;
        if (nblocks > 0x7fffffffL) return set_err(c, SPARC_ERR_ARG, "too many blocks");
        k_proj_stream<T><<<dim3((unsigned)nblocks), 64 * a.nw, shmem, stream>>>(x + (long)c0 * ldx, a);
        SG_CHECK_LAUNCH(c);
        k_proj_reduce<T><<<dim3(c->n_atoms, div_up(4L * a.ncol, 256)), 256, 0, stream>>>(
            part, a.ncol, a.zsplit, (long)a.ntiles_y * a.kmax, NT.red_off, NT.red_idx, NT.gamma4, c->dV,
            D_of<T>(c) + (long)c0 * 4 * c->n_atoms, 4 * c->n_atoms);
        SG_CHECK_LAUNCH(c);
    }
    prof_end(c, slot, stream);
    return SPARC_OK;
}

template sparc_status launch_hsweep<double>(sparc_gpu_ctx, const double*, double*, const double*, int, long, int,
                                            int);
template sparc_status launch_hsweep<float>(sparc_gpu_ctx, const float*, float*, const float*, int, long, int, int);
template sparc_status launch_projection<double>(sparc_gpu_ctx, const double*, int, long, double*, size_t);
template sparc_status launch_projection<float>(sparc_gpu_ctx, const float*, int, long, double*, size_t);

// ---- allocation-free filter -----------------------------------------------
// The projection partials of sparc_gpu_chebyshev_filter_noalloc live in this
// fixed array (32 MiB; each GPU the library runs on holds its own copy until
// the process ends) instead of memory the library allocates.  Host code never
// names the array: it uses the device address looked up once per device by
// scratch_init.  Calls that overlap on one GPU share it and race.
constexpr size_t kScratchDoubles = (size_t)4 << 20;
static __device__ __align__(256) double scratch[kScratchDoubles];

sparc_status scratch_init(sparc_gpu_ctx c, int dev) {
    static std::mutex mu;
    static std::map<int, double*> addr;   // device -> address of its copy of the array
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_err(c, e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
        it = addr.emplace(dev, static_cast<double*>(ptr)).first;
    }
    c->scratch = it->second;
    c->scratch_elems = kScratchDoubles;
    return SPARC_OK;
}

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
// even and in W when k is odd; the result ends in X.  Before each sweep the
// projection pass forms the projections of its operand Y_{k-1}.
template <typename T>
sparc_status filter_impl(sparc_gpu_ctx c, T* X, T* Wk, int ncol, long ldx, int m, double* part, size_t part_elems) {
    sparc_status st;
    // every sweep needs the projections of its operand
    if ((st = launch_projection<T>(c, X, ncol, ldx, part, part_elems)) != SPARC_OK) return st;
    if ((st = launch_hsweep<T>(c, X, Wk, nullptr, ncol, ldx, 1, 1)) != SPARC_OK) return st;
    for (int k = 2; k <= m; ++k) {
        T* cur = (k % 2 == 0) ? Wk : X;   // Y_{k-1}
        T* dst = (k % 2 == 0) ? X : Wk;   // Y_{k-2}, overwritten with Y_k
        if ((st = launch_projection<T>(c, cur, ncol, ldx, part, part_elems)) != SPARC_OK) return st;
        if ((st = launch_hsweep<T>(c, cur, dst, dst, ncol, ldx, 2, k)) != SPARC_OK) return st;
    }
    if (m % 2 == 1) {
        dim3 grid(div_up(c->nd, 256), ncol);
        const int slot = prof_begin(c, PK_COPY);
        k_copy_block<T><<<grid, 256, 0, c->stream>>>(Wk, X, c->nd, ncol, ldx);
        SG_CHECK_LAUNCH(c);
        prof_end(c, slot);
    }
    return SPARC_OK;
}

template sparc_status filter_impl<double>(sparc_gpu_ctx, double*, double*, int, long, int, double*, size_t);
template sparc_status filter_impl<float>(sparc_gpu_ctx, float*, float*, int, long, int, double*, size_t);

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

sparc_status sparc_gpu_chebyshev_filter_noalloc(sparc_gpu_ctx c, sparc_prec prec, void* d_X, void* d_work, int ncol,
                                                long ldx, int degree, double a, double b, double a0) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    sparc_status st = check_block(c, prec, d_X, ncol, ldx, "chebyshev_filter_noalloc");
    if (st != SPARC_OK) return st;
    if (!d_work) return set_err(c, SPARC_ERR_ARG, "chebyshev_filter_noalloc: null work block");
    if (degree < 1 || degree > 10000) return set_err(c, SPARC_ERR_ARG, "chebyshev_filter_noalloc: degree out of range");
    if (!(a0 < a && a < b) || !std::isfinite(a0) || !std::isfinite(b))
        return set_err(c, SPARC_ERR_ARG, "chebyshev_filter_noalloc: need a0 < a < b");
    size_t es = prec == SPARC_FP64 ? 8 : 4;
    size_t bytes = ((size_t)(ncol - 1) * ldx + c->nd) * es;
    if (overlaps(d_X, d_work, bytes)) return set_err(c, SPARC_ERR_ARG, "chebyshev_filter_noalloc: X and work overlap");
    if (!c->scratch) return set_err(c, SPARC_ERR_ARG, "chebyshev_filter_noalloc: no scratch array on this device");
    k_set3<<<1, 1, 0, c->stream>>>(c->scal + S_A, a, b, a0);
    SG_CHECK_LAUNCH(c);
    // no timing events either (creating them could allocate)
    const bool prof = c->prof;
    c->prof = false;
    const sparc_status r =
        prec == SPARC_FP64
            ? filter_impl<double>(c, (double*)d_X, (double*)d_work, ncol, ldx, degree, c->scratch, c->scratch_elems)
            : filter_impl<float>(c, (float*)d_X, (float*)d_work, ncol, ldx, degree, c->scratch, c->scratch_elems);
    c->prof = prof;
    return r;
}

}  // extern "C"
