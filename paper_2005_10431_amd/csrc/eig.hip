// Dense symmetric eigensolver of the Rayleigh-Ritz step (FP64): Householder
// reduction to tridiagonal form, eigenvalues by Sturm-sequence bisection,
// eigenvectors by inverse iteration (re-orthogonalised inside clusters of
// close eigenvalues), and back-transformation by the Householder
// reflectors.  These are the textbook steps of a tridiagonal-based symmetric
// eigensolver; the Ns x Ns problem is the part of CheFSI whose cubic cost the
// paper names as its scaling limit (Sec. 4).
//
// All matrices are N x N column-major with leading dimension N.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "internal.hpp"

namespace sg {

constexpr double kEps = 2.220446049250313e-16;

__device__ inline double block_sum(double v, double* red) {
    // blockDim.x is a multiple of 64 and <= 1024
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];  // fixed order
    return s;
}

// Householder tridiagonalisation (lower), one workgroup, of A - sigma I with
// sigma = trace(A)/N (the shift keeps ||T|| at the spread of the spectrum,
// which is what the cluster test of the inverse iteration measures against).
// On exit d, e hold the tridiagonal matrix, column i of A below the
// subdiagonal holds the reflector v_i (v_i[i+1] = 1 implicit), tau[i] its
// factor, and shift[0] = sigma:
//   H_i = I - tau_i v v^T,  Q = H_0 H_1 ... H_{N-3},  Q^T (A - sigma I) Q = T.
// Each step reads and writes the trailing matrix once: the rank-2 update of
// step i is fused with the product A v_{i+1} of step i+1 (the next reflector
// comes from the updated column i+1, which is updated first).
struct TrdLayout {
    int rows, R, G, TPG;
};

__device__ inline TrdLayout trd_layout(int rows, int nt) {
    TrdLayout L;
    L.rows = rows;
    L.R = ((rows + 63) / 64) * 64;
    L.G = max(1, min(16, nt / max(L.R, 64)));
    L.TPG = ((nt / L.G) / 64) * 64;
    return L;
}

// Householder vector of x = A[j+1 .., j] (length N-j-1) into vn (indexed by
// global row), returns tau, writes beta to *beta_out.  All threads call it.
__device__ inline double trd_householder(double* A, int N, int j, double* vn, double* red, double* beta_out) {
    const int t = threadIdx.x, nt = blockDim.x;
    const double* x = A + (long)j * N;
    double s = 0.0;
    for (int r = j + 2 + t; r < N; r += nt) s += x[r] * x[r];
    const double xnorm2 = block_sum(s, red);
    const double alpha = x[j + 1];
    double tau = 0.0, beta = alpha;
    if (xnorm2 > 0.0) {
        beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
        tau = (beta - alpha) / beta;
    }
    const double scal = (xnorm2 > 0.0) ? 1.0 / (alpha - beta) : 0.0;
    for (int r = j + 1 + t; r < N; r += nt) vn[r] = (r == j + 1) ? 1.0 : x[r] * scal;
    *beta_out = beta;
    return tau;
}

// Trailing pass over rows/cols >= lo: optionally apply A -= v w^T + w v^T,
// and accumulate acc[g] = sum_h A[g,h] vn[h] into part[] (G groups).
template <bool UPDATE>
__device__ inline void trd_pass(double* A, int N, int lo, const double* v, const double* w, const double* vn,
                                double* part, TrdLayout L) {
    const int t = threadIdx.x;
    const int grp = t / L.TPG;
    if (grp >= L.G) return;
    const int lr0 = t - grp * L.TPG;
    for (int lr = lr0; lr < L.rows; lr += L.TPG) {
        const int g = lo + lr;
        const double vg = UPDATE ? v[g] : 0.0, wg = UPDATE ? w[g] : 0.0;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int h = lo + grp;
        const int G = L.G;
        for (; h + 3 * G < N; h += 4 * G) {
            double* p0 = A + g + (long)h * N;
            double x0 = p0[0], x1 = p0[(long)G * N], x2 = p0[(long)2 * G * N], x3 = p0[(long)3 * G * N];
            if (UPDATE) {
                x0 -= vg * w[h] + wg * v[h];
                x1 -= vg * w[h + G] + wg * v[h + G];
                x2 -= vg * w[h + 2 * G] + wg * v[h + 2 * G];
                x3 -= vg * w[h + 3 * G] + wg * v[h + 3 * G];
                p0[0] = x0;
                p0[(long)G * N] = x1;
                p0[(long)2 * G * N] = x2;
                p0[(long)3 * G * N] = x3;
            }
            a0 += x0 * vn[h];
            a1 += x1 * vn[h + G];
            a2 += x2 * vn[h + 2 * G];
            a3 += x3 * vn[h + 3 * G];
        }
        for (; h < N; h += G) {
            double* p0 = A + g + (long)h * N;
            double x0 = p0[0];
            if (UPDATE) {
                x0 -= vg * w[h] + wg * v[h];
                p0[0] = x0;
            }
            a0 += x0 * vn[h];
        }
        part[grp * L.R + lr] = (a0 + a1) + (a2 + a3);
    }
}

// Steps i0, i0+1, ..., N-3 of the reduction, then the last diagonal and
// subdiagonal entries.  On entry v (LDS, global row index) holds reflector
// i0 with factor tau_i, and A[i0+1:, i0+1:] is updated through step i0-1.
__device__ inline void trd_run(double* A, int N, int i0, double* v, double* w, double* vn, double* part,
                               double tau_i, double* d, double* e, double* tau, double* red, double* sbeta) {
    const int t = threadIdx.x, nt = blockDim.x;
    TrdLayout L = trd_layout(N - (i0 + 1), nt);
    trd_pass<false>(A, N, i0 + 1, v, w, v, part, L);
    __syncthreads();
    for (int i = i0; i + 2 < N; ++i) {
        // p = tau A22 v from the partial sums, rows g >= i+1
        const int lo = i + 1;
        double pv = 0.0;
        for (int lr = t; lr < L.rows; lr += nt) {
            double acc = 0.0;
            for (int q = 0; q < L.G; ++q) acc += part[q * L.R + lr];
            const double p = tau_i * acc;
            w[lo + lr] = p;
            pv += p * v[lo + lr];
        }
        pv = block_sum(pv, red);
        const double k2 = 0.5 * tau_i * pv;
        for (int g = lo + t; g < N; g += nt) w[g] -= k2 * v[g];
        __syncthreads();
        // reflector i is stored below the subdiagonal of column i
        {
            double* x = A + (long)i * N;
            for (int r = i + 2 + t; r < N; r += nt) x[r] = v[r];
        }
        const bool more = (i + 1) + 2 < N;
        const int h = i + 1;
        double* col = A + (long)h * N;
        const double vh = v[h], wh = w[h];
        double tau_n = 0.0;
        if (more) {
            // column i+1 (rows >= i+1) is updated in registers and yields
            // the next reflector directly: its diagonal is d[i+1], row
            // i+2 is alpha, rows >= i+3 the rest of x
            double cv[4];  // N <= 4 nt
            double ss = 0.0;
            int q = 0;
            for (int g = h + t; g < N; g += nt, ++q) {
                const double val = col[g] - (v[g] * wh + w[g] * vh);
                cv[q] = val;
                if (g == h) d[h] = val;
                if (g == h + 1) *sbeta = val;  // alpha, read after the reduction's barriers
                if (g >= h + 2) ss += val * val;
            }
            const double xnorm2 = block_sum(ss, red);
            const double alpha = *sbeta;
            double bn = alpha;
            if (xnorm2 > 0.0) {
                bn = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
                tau_n = (bn - alpha) / bn;
            }
            const double scal = (xnorm2 > 0.0) ? 1.0 / (alpha - bn) : 0.0;
            q = 0;
            for (int g = h + t; g < N; g += nt, ++q) {
                if (g == h + 1) {
                    vn[g] = 1.0;
                } else if (g >= h + 2) {
                    const double vv = cv[q] * scal;
                    vn[g] = vv;
                    col[g] = vv;
                }
            }
            if (t == 0) {
                e[h] = bn;
                tau[h] = tau_n;
            }
        } else {
            // last step: the updated column gives the final d and e
            for (int g = h + t; g < N; g += nt) col[g] -= v[g] * wh + w[g] * vh;
            for (int g = t; g < N; g += nt) vn[g] = 0.0;
        }
        __syncthreads();
        L = trd_layout(N - (i + 2), nt);
        trd_pass<true>(A, N, i + 2, v, w, vn, part, L);
        __syncthreads();
        if (!more) break;
        double* tmp = v;
        v = vn;
        vn = tmp;
        tau_i = tau_n;
    }
}

__device__ inline void trd_final(const double* A, int N, double* d, double* e, double* tau) {
    if (threadIdx.x == 0) {
        if (N >= 2) {
            d[N - 2] = A[(N - 2) + (long)(N - 2) * N];
            e[N - 2] = A[(N - 1) + (long)(N - 2) * N];
            tau[N - 2] = 0.0;
        }
        d[N - 1] = A[(N - 1) + (long)(N - 1) * N];
    }
}

__global__ __launch_bounds__(1024) void k_sytrd(double* A, int N, double* d, double* e, double* tau, double* shift) {
    extern __shared__ double sh[];
    double* v = sh;             // N: current reflector (global row index)
    double* w = sh + N;         // N
    double* vn = sh + 2 * N;    // N: next reflector
    double* part = sh + 3 * N;  // <= 1024 + 16 * 64 partial sums
    __shared__ double red[16];
    __shared__ double s_beta;
    const int t = threadIdx.x, nt = blockDim.x;
    // shift by the mean of the diagonal
    double tr = 0.0;
    for (int i = t; i < N; i += nt) tr += A[i + (long)i * N];
    const double sigma = block_sum(tr, red) / N;
    __syncthreads();
    for (int i = t; i < N; i += nt) A[i + (long)i * N] -= sigma;
    if (t == 0) shift[0] = sigma;
    __syncthreads();
    if (N >= 3) {
        double beta;
        const double tau0 = trd_householder(A, N, 0, v, red, &beta);
        if (t == 0) {
            d[0] = A[0];
            e[0] = beta;
            tau[0] = tau0;
        }
        __syncthreads();
        trd_run(A, N, 0, v, w, vn, part, tau0, d, e, tau, red, &s_beta);
    }
    trd_final(A, N, d, e, tau);
}

// The last steps of the many-workgroup reduction, from step i0 on, in one
// workgroup: vg holds reflector i0 (global row index), sc[i0 & 1] its tau.
__global__ __launch_bounds__(1024) void k_sytrd_tail(double* A, int N, int i0, const double* __restrict__ vg,
                                                     const double* __restrict__ sc, double* d, double* e,
                                                     double* tau) {
    extern __shared__ double sh[];
    double* v = sh;
    double* w = sh + N;
    double* vn = sh + 2 * N;
    double* part = sh + 3 * N;
    __shared__ double red[16];
    __shared__ double s_beta;
    for (int r = i0 + 1 + threadIdx.x; r < N; r += blockDim.x) v[r] = vg[r];
    const double tau_i = sc[i0 & 1];
    __syncthreads();
    trd_run(A, N, i0, v, w, vn, part, tau_i, d, e, tau, red, &s_beta);
    trd_final(A, N, d, e, tau);
}

// ---- the same reduction over many workgroups (large N) ---------------------
// Each step is two launches: one workgroup turns the per-block partial
// products of the previous pass into w, stores the reflector and forms the
// next reflector from the updated next column (as k_sytrd does); then a grid
// of (64-row x 128-column) tiles applies the rank-2 update to the trailing
// matrix and forms the partial products with the next reflector, one
// partial per (column tile, row), summed in tile order by the next step.

constexpr int kTrdRB = 64;   // rows per pass workgroup (one wave's lanes)
constexpr int kTrdCB = 128;  // columns per pass workgroup
constexpr int kTrdCG = 16;  // waves per pass workgroup, each a column stride
constexpr int kTrdCW = kTrdCB / kTrdCG;  // columns per wave
static_assert(kTrdCB % kTrdCG == 0, "pass tile width must split evenly over its waves");
static_assert(kEighMaxN <= 4 * 1024, "k_trd_step and trd_run hold at most 4 rows per thread of 1024");

__global__ __launch_bounds__(1024) void k_trd_first(double* A, int N, double* d, double* e, double* tau,
                                                    double* shift, double* v, double* sc) {
    __shared__ double red[16];
    const int t = threadIdx.x, nt = blockDim.x;
    double tr = 0.0;
    for (int i = t; i < N; i += nt) tr += A[i + (long)i * N];
    const double sigma = block_sum(tr, red) / N;
    __syncthreads();
    for (int i = t; i < N; i += nt) A[i + (long)i * N] -= sigma;
    __syncthreads();
    double beta;
    const double tau0 = trd_householder(A, N, 0, v, red, &beta);
    if (t == 0) {
        shift[0] = sigma;
        d[0] = A[0];
        e[0] = beta;
        tau[0] = tau0;
        sc[0] = tau0;
    }
}

// Rows [lo, N) x columns of tile blockIdx.x: optional rank-2 update
// A -= v w^T + w v^T, and part[tile][g] = sum over the tile's columns of
// A[g, h] vn[h] (wave partials summed in wave order).
template <bool UPDATE>
__global__ __launch_bounds__(1024) void k_trd_pass_multi(double* A, int N, int lo, const double* __restrict__ v,
                                                         const double* __restrict__ w,
                                                         const double* __restrict__ vn, double* __restrict__ part) {
    __shared__ double red[kTrdCG][kTrdRB];
    const int lane = threadIdx.x & 63, cg = threadIdx.x >> 6;
    const int g = lo + blockIdx.y * kTrdRB + lane;
    const int hb = lo + blockIdx.x * kTrdCB;
    const int he = min(N, hb + kTrdCB);
    double acc = 0.0;
    if (g < N) {
        const double vg = UPDATE ? v[g] : 0.0, wg = UPDATE ? w[g] : 0.0;
#pragma unroll
        for (int j = 0; j < kTrdCW; ++j) {
            const int h = hb + cg + j * kTrdCG;
            if (h < he) {
                double* p = A + g + (long)h * N;
                double x = *p;
                if (UPDATE) {
                    x -= vg * w[h] + wg * v[h];
                    *p = x;
                }
                acc += x * vn[h];
            }
        }
    }
    red[cg][lane] = acc;
    __syncthreads();
    if (cg == 0 && g < N) {
        double sum = 0.0;
        for (int q = 0; q < kTrdCG; ++q) sum += red[q][lane];
        part[(long)blockIdx.x * N + g] = sum;
    }
}

// Step i: p = tau A22 v from the nbp partial tiles, w = p - (tau/2)(p.v) v,
// reflector i into column i, column i+1 updated and turned into the next
// reflector vn (or, on the last step, just updated).  sc[i & 1] holds the
// tau of v, sc[(i + 1) & 1] receives that of vn.
__global__ __launch_bounds__(1024) void k_trd_step(double* A, int N, int i, int nbp, const double* __restrict__ part,
                                                   const double* __restrict__ v, double* __restrict__ w,
                                                   double* __restrict__ vn, double* d, double* e, double* tau,
                                                   double* sc) {
    __shared__ double red[16];
    __shared__ double s_wh, s_beta;
    const int t = threadIdx.x, nt = blockDim.x;
    const int h = i + 1;  // first row of the trailing block, and the next column
    const double tau_i = sc[i & 1];
    double* col = A + (long)h * N;
    double* x = A + (long)i * N;
    // rows g = h + t + q nt (N <= 4 nt): every load up front
    double vg[4], wg[4], cg[4];
    double pv = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int g = h + t + q * nt;
        vg[q] = wg[q] = cg[q] = 0.0;
        if (g < N) {
            vg[q] = v[g];
            cg[q] = col[g];
            double acc = 0.0;
            for (int b = 0; b < nbp; ++b) acc += part[(long)b * N + g];
            wg[q] = tau_i * acc;
            pv += wg[q] * vg[q];
            if (g >= i + 2) x[g] = vg[q];  // reflector i below the subdiagonal of column i
        }
    }
    pv = block_sum(pv, red);
    const double k2 = 0.5 * tau_i * pv;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int g = h + t + q * nt;
        if (g < N) {
            wg[q] -= k2 * vg[q];
            w[g] = wg[q];
            if (g == h) s_wh = wg[q];
        }
    }
    __syncthreads();
    const double wh = s_wh, vh = v[h];
    if (h + 2 < N) {
        double ss = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int g = h + t + q * nt;
            if (g < N) {
                const double val = cg[q] - (vg[q] * wh + wg[q] * vh);
                cg[q] = val;
                if (g == h) d[h] = val;
                if (g == h + 1) s_beta = val;
                if (g >= h + 2) ss += val * val;
            }
        }
        const double xnorm2 = block_sum(ss, red);
        const double alpha = s_beta;
        double bn = alpha, tau_n = 0.0;
        if (xnorm2 > 0.0) {
            bn = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
            tau_n = (bn - alpha) / bn;
        }
        const double scal = (xnorm2 > 0.0) ? 1.0 / (alpha - bn) : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int g = h + t + q * nt;
            if (g == h + 1) {
                vn[g] = 1.0;
            } else if (g >= h + 2 && g < N) {
                const double vv = cg[q] * scal;
                vn[g] = vv;
                col[g] = vv;
            }
        }
        if (t == 0) {
            e[h] = bn;
            tau[h] = tau_n;
            sc[(i + 1) & 1] = tau_n;
        }
    } else {
        // last step: the updated column gives the final d and e
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int g = h + t + q * nt;
            if (g < N) col[g] = cg[q] - (vg[q] * wh + wg[q] * vh);
        }
        for (int g = t; g < N; g += nt) vn[g] = 0.0;
    }
}

__global__ void k_trd_final(const double* A, int N, double* d, double* e, double* tau) {
    trd_final(A, N, d, e, tau);
}

// The k_sytrd reduction with the trailing passes spread over the chip; once
// the trailing matrix has at most `tail` rows, one workgroup (k_sytrd_tail)
// takes the remaining steps.  scratch: 3 N + 8 + ceil(N / kTrdCB) N doubles.
// N >= 3.
static sparc_status sytrd_multi(sparc_gpu_ctx c, double* A, int N, int tail, double* d, double* e, double* tau,
                                double* shift, double* scratch) {
    double* v = scratch;
    double* w = v + N;
    double* vn = w + N;
    double* sc = vn + N;
    double* part = sc + 8;
    const int threads = std::min(1024, std::max(64, div_up(N, 64) * 64));
    k_trd_first<<<1, threads, 0, c->stream>>>(A, N, d, e, tau, shift, v, sc);
    SG_CHECK_LAUNCH(c);
    const int pass_threads = 64 * kTrdCG;
    if (N - 1 > tail) {
        const int m = N - 1;
        const dim3 grid(div_up(m, kTrdCB), div_up(m, kTrdRB));
        k_trd_pass_multi<false><<<grid, pass_threads, 0, c->stream>>>(A, N, 1, v, w, v, part);
        SG_CHECK_LAUNCH(c);
    }
    int i = 0;
    bool done = false;
    for (; i + 2 < N; ++i) {
        if (N - (i + 1) <= tail) break;
        const int nbp = div_up(N - (i + 1), kTrdCB);
        k_trd_step<<<1, threads, 0, c->stream>>>(A, N, i, nbp, part, v, w, vn, d, e, tau, sc);
        const int lo = i + 2, m = N - lo;
        if (m > 0) {
            const dim3 grid(div_up(m, kTrdCB), div_up(m, kTrdRB));
            k_trd_pass_multi<true><<<grid, pass_threads, 0, c->stream>>>(A, N, lo, v, w, vn, part);
        }
        SG_CHECK_LAUNCH(c);
        if (i + 3 >= N) {
            done = true;
            break;
        }
        std::swap(v, vn);
    }
    if (done) {
        k_trd_final<<<1, 64, 0, c->stream>>>(A, N, d, e, tau);
    } else {
        const size_t lds = (3 * (size_t)N + std::max(1024, N + 64)) * sizeof(double);
        k_sytrd_tail<<<1, threads, lds, c->stream>>>(A, N, i, v, sc, d, e, tau);
    }
    SG_CHECK_LAUNCH(c);
    return SPARC_OK;
}

// Number of eigenvalues of T smaller than x (Sturm count of the LDL^T
// pivots of T - x I).
__device__ inline int sturm_count(const double* d, const double* e2, int N, double x, double pivmin) {
    int cnt = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++cnt;
    for (int i = 1; i < N; ++i) {
        q = d[i] - x - e2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

// k-th smallest eigenvalue of T (workgroup k of 64 lanes): multisection of
// the Gershgorin interval, 64 Sturm counts per round.  lam gets the
// eigenvalue of T, eig the eigenvalue of A (T + shift).
__global__ __launch_bounds__(64) void k_bisect(const double* d, const double* e, int N, const double* shift,
                                               double* lam, double* eig) {
    extern __shared__ double sh[];
    double* sd = sh;
    double* se2 = sh + N;
    const int k = blockIdx.x, lane = threadIdx.x;
    double lo = 1e300, hi = -1e300, emax2 = 0.0, tnorm = 0.0;
    for (int i = lane; i < N; i += 64) {
        const double di = d[i];
        const double el = (i > 0) ? fabs(e[i - 1]) : 0.0, er = (i + 1 < N) ? fabs(e[i]) : 0.0;
        sd[i] = di;
        se2[i] = er * er;
        lo = fmin(lo, di - el - er);
        hi = fmax(hi, di + el + er);
        tnorm = fmax(tnorm, fabs(di) + el + er);
        emax2 = fmax(emax2, er * er);
    }
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
        tnorm = fmax(tnorm, __shfl_xor(tnorm, off, 64));
        emax2 = fmax(emax2, __shfl_xor(emax2, off, 64));
    }
    __syncthreads();
    const double pad = 2.0 * kEps * tnorm * N + 1e-300;
    lo -= pad;
    hi += pad;
    const double pivmin = 1e-290 * fmax(1.0, emax2);
    for (int it = 0; it < 64; ++it) {
        if (!(hi - lo > 2.0 * kEps * fmax(fabs(lo), fabs(hi)) + 1e-300)) break;
        const double x = lo + (hi - lo) * ((double)(lane + 1) / 65.0);
        const bool above = (x > lo && x < hi) ? (sturm_count(sd, se2, N, x, pivmin) > k) : (x >= hi);
        const unsigned long long m = __ballot(above);
        // first lane whose point has more than k eigenvalues below it
        const int j = m ? __ffsll((long long)m) - 1 : 64;
        const double nlo = (j == 0) ? lo : __shfl(x, j - 1 < 0 ? 0 : j - 1, 64);
        const double nhi = (j == 64) ? hi : __shfl(x, j > 63 ? 63 : j, 64);
        if (!(nlo >= lo && nhi <= hi && nlo < nhi) || (nlo == lo && nhi == hi)) break;
        lo = nlo;
        hi = nhi;
    }
    if (lane == 0) {
        const double l = 0.5 * (lo + hi);
        lam[k] = l;
        eig[k] = l + shift[0];
    }
}

// Start vector of inverse iteration for eigenvalue k: a fixed,
// index-dependent pattern in [0.5, 1.5) (a low-discrepancy sequence; any
// vector with a component along the wanted eigenvector works).
__device__ inline double start_value(int i, int k) {
    const double u = i * 0.6180339887498949 + (k + 1) * 0.7548776662466927;
    return 0.5 + (u - floor(u));
}

// Inverse iteration for the eigenvectors of T, one thread per cluster of
// close eigenvalues (consecutive indices whose gaps are below 1e-5 ||T||);
// members of a cluster are shifted apart by a few ulps and Gram-Schmidt
// orthogonalised against the earlier members at every step.  Scratch is
// interleaved by thread (element i of thread c at i * nthr + c) so that a
// wave's accesses coalesce; the vectors go to zt (row k = eigenvector k,
// element i at i * N + k, i.e. zt is Z^T in column-major order).
__global__ __launch_bounds__(64) void k_stein(const double* d, const double* e, const double* lam, int N,
                                              const int* cl_start, const int* ncl, double* zt, double* work) {
    const int nthr = gridDim.x * blockDim.x;
    const int cl = blockIdx.x * blockDim.x + threadIdx.x;
    if (cl >= *ncl) return;
    const int k0 = cl_start[cl], k1 = cl_start[cl + 1];
    double* lo = work;                       // multiplier of L
    double* rd = lo + (long)N * nthr;        // 1 / diagonal of U
    double* u1 = rd + (long)N * nthr;        // first superdiagonal of U
    double* u2 = u1 + (long)N * nthr;        // second superdiagonal of U (pivoting)
    double* pv = u2 + (long)N * nthr;        // +1 where rows i, i+1 were interchanged
#define SG_AT(arr, i) arr[(long)(i) * nthr + cl]
#define SG_Z(i, k) zt[(long)(i) * N + (k)]
    double tnorm = 0.0;
    for (int i = 0; i < N; ++i)
        tnorm = fmax(tnorm, fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < N ? fabs(e[i]) : 0.0));
    // floor keeps 1/tiny^2 finite for a (near-)zero T
    const double tiny = kEps * fmax(tnorm, 1e-100);
    const double sep = 10.0 * tiny;
    double prev = -1e300;
    for (int k = k0; k < k1; ++k) {
        double x = lam[k];
        if (k > k0 && x - prev < sep) x = prev + sep;
        prev = x;
        // LU with partial pivoting of T - x I (one reciprocal per pivot)
        double a = d[0] - x, b = (N > 1) ? e[0] : 0.0;
        for (int i = 0; i < N - 1; ++i) {
            const double c = e[i];
            const double dn = d[i + 1] - x;
            const double bn = (i + 2 < N) ? e[i + 1] : 0.0;
            if (fabs(a) >= fabs(c)) {
                if (fabs(a) < tiny) a = (a < 0.0) ? -tiny : tiny;
                const double r = 1.0 / a;
                const double l = c * r;
                SG_AT(lo, i) = l;
                SG_AT(rd, i) = r;
                SG_AT(u1, i) = b;
                SG_AT(u2, i) = 0.0;
                SG_AT(pv, i) = 0.0;
                a = dn - l * b;
                b = bn;
            } else {
                const double r = 1.0 / c;
                const double l = a * r;
                SG_AT(lo, i) = l;
                SG_AT(rd, i) = r;
                SG_AT(u1, i) = dn;
                SG_AT(u2, i) = bn;
                SG_AT(pv, i) = 1.0;
                a = b - l * dn;
                b = -l * bn;
            }
        }
        if (fabs(a) < tiny) a = (a < 0.0) ? -tiny : tiny;
        SG_AT(rd, N - 1) = 1.0 / a;
        for (int i = 0; i < N; ++i) SG_Z(i, k) = start_value(i, k);
        for (int it = 0; it < 4; ++it) {
            // forward: apply the row interchanges and L^{-1}; the operands of
            // CH steps are loaded before the chain that consumes them
            constexpr int CH = 8;
            double cur = SG_Z(0, k);
            int i = 0;
            for (; i + CH <= N - 1; i += CH) {
                double nz[CH], l[CH], pq[CH];
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    nz[u] = SG_Z(i + u + 1, k);
                    l[u] = SG_AT(lo, i + u);
                    pq[u] = SG_AT(pv, i + u);
                }
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    if (pq[u] != 0.0) {
                        SG_Z(i + u, k) = nz[u];
                        cur = cur - l[u] * nz[u];
                    } else {
                        SG_Z(i + u, k) = cur;
                        cur = nz[u] - l[u] * cur;
                    }
                }
            }
            for (; i < N - 1; ++i) {
                const double nxt = SG_Z(i + 1, k);
                const double l = SG_AT(lo, i);
                if (SG_AT(pv, i) != 0.0) {
                    SG_Z(i, k) = nxt;
                    cur = cur - l * nxt;
                } else {
                    SG_Z(i, k) = cur;
                    cur = nxt - l * cur;
                }
            }
            // backward: U^{-1}
            double x1 = cur * SG_AT(rd, N - 1), x2 = 0.0;
            SG_Z(N - 1, k) = x1;
            i = N - 2;
            for (; i - (CH - 1) >= 0; i -= CH) {
                double zv[CH], a1[CH], a2[CH], r[CH];
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    zv[u] = SG_Z(i - u, k);
                    a1[u] = SG_AT(u1, i - u);
                    a2[u] = SG_AT(u2, i - u);
                    r[u] = SG_AT(rd, i - u);
                }
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    const double xi = (zv[u] - a1[u] * x1 - a2[u] * x2) * r[u];
                    SG_Z(i - u, k) = xi;
                    x2 = x1;
                    x1 = xi;
                }
            }
            for (; i >= 0; --i) {
                const double xi = (SG_Z(i, k) - SG_AT(u1, i) * x1 - SG_AT(u2, i) * x2) * SG_AT(rd, i);
                SG_Z(i, k) = xi;
                x2 = x1;
                x1 = xi;
            }
            // orthogonalise against earlier members of the cluster, normalise
            for (int j = k0; j < k; ++j) {
                double s = 0.0;
                for (int i = 0; i < N; ++i) s += SG_Z(i, j) * SG_Z(i, k);
                for (int i = 0; i < N; ++i) SG_Z(i, k) -= s * SG_Z(i, j);
            }
            double nrm = 0.0;
            for (int i = 0; i < N; ++i) nrm += SG_Z(i, k) * SG_Z(i, k);
            const double inv = (nrm > 0.0) ? 1.0 / sqrt(nrm) : 0.0;
            for (int i = 0; i < N; ++i) SG_Z(i, k) *= inv;
        }
    }
#undef SG_AT
#undef SG_Z
}

// Same inverse iteration with every thread's factors and vector in LDS
// (tpw threads per workgroup, element i of lane l at i * tpw + l; d and e
// shared).  Used when 6 N tpw + 2 N doubles fit in LDS.
__global__ __launch_bounds__(64) void k_stein_lds(const double* d, const double* e, const double* lam, int N,
                                                  const int* cl_start, const int* ncl, double* zt, int tpw) {
    extern __shared__ double sh[];
    double* sd = sh;                        // N
    double* se = sh + N;                    // N
    double* lo = se + N;                    // multiplier of L
    double* rd = lo + (long)N * tpw;        // 1 / diagonal of U
    double* u1 = rd + (long)N * tpw;        // first superdiagonal of U
    double* u2 = u1 + (long)N * tpw;        // second superdiagonal of U (pivoting)
    double* pv = u2 + (long)N * tpw;        // +1 where rows i, i+1 were interchanged
    double* z = pv + (long)N * tpw;         // the vector being iterated
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        sd[i] = d[i];
        se[i] = (i + 1 < N) ? e[i] : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x;
    const int cl = blockIdx.x * tpw + lane;
    if (lane >= tpw || cl >= *ncl) return;  // no barrier below
#define SG_L(arr, i) arr[(long)(i) * tpw + lane]
    const int k0 = cl_start[cl], k1 = cl_start[cl + 1];
    double tnorm = 0.0;
    for (int i = 0; i < N; ++i)
        tnorm = fmax(tnorm, fabs(sd[i]) + (i > 0 ? fabs(se[i - 1]) : 0.0) + (i + 1 < N ? fabs(se[i]) : 0.0));
    const double tiny = kEps * fmax(tnorm, 1e-100);
    const double sep = 10.0 * tiny;
    double prev = -1e300;
    for (int k = k0; k < k1; ++k) {
        double x = lam[k];
        if (k > k0 && x - prev < sep) x = prev + sep;
        prev = x;
        double a = sd[0] - x, b = (N > 1) ? se[0] : 0.0;
        for (int i = 0; i < N - 1; ++i) {
            const double c = se[i];
            const double dn = sd[i + 1] - x;
            const double bn = se[i + 1];
            if (fabs(a) >= fabs(c)) {
                if (fabs(a) < tiny) a = (a < 0.0) ? -tiny : tiny;
                const double r = 1.0 / a;
                const double l = c * r;
                SG_L(lo, i) = l;
                SG_L(rd, i) = r;
                SG_L(u1, i) = b;
                SG_L(u2, i) = 0.0;
                SG_L(pv, i) = 0.0;
                a = dn - l * b;
                b = bn;
            } else {
                const double r = 1.0 / c;
                const double l = a * r;
                SG_L(lo, i) = l;
                SG_L(rd, i) = r;
                SG_L(u1, i) = dn;
                SG_L(u2, i) = bn;
                SG_L(pv, i) = 1.0;
                a = b - l * dn;
                b = -l * bn;
            }
        }
        if (fabs(a) < tiny) a = (a < 0.0) ? -tiny : tiny;
        SG_L(rd, N - 1) = 1.0 / a;
        for (int i = 0; i < N; ++i) SG_L(z, i) = start_value(i, k);
        for (int it = 0; it < 4; ++it) {
            double cur = SG_L(z, 0);
            for (int i = 0; i < N - 1; ++i) {
                const double nxt = SG_L(z, i + 1);
                const double l = SG_L(lo, i);
                if (SG_L(pv, i) != 0.0) {
                    SG_L(z, i) = nxt;
                    cur = cur - l * nxt;
                } else {
                    SG_L(z, i) = cur;
                    cur = nxt - l * cur;
                }
            }
            double x1 = cur * SG_L(rd, N - 1), x2 = 0.0;
            SG_L(z, N - 1) = x1;
            for (int i = N - 2; i >= 0; --i) {
                const double xi = (SG_L(z, i) - SG_L(u1, i) * x1 - SG_L(u2, i) * x2) * SG_L(rd, i);
                SG_L(z, i) = xi;
                x2 = x1;
                x1 = xi;
            }
            // orthogonalise against the earlier members of the cluster
            // (already written to zt by this thread), normalise
            for (int j = k0; j < k; ++j) {
                double s = 0.0;
                for (int i = 0; i < N; ++i) s += zt[(long)i * N + j] * SG_L(z, i);
                for (int i = 0; i < N; ++i) SG_L(z, i) -= s * zt[(long)i * N + j];
            }
            double nrm = 0.0;
            for (int i = 0; i < N; ++i) nrm += SG_L(z, i) * SG_L(z, i);
            const double inv = (nrm > 0.0) ? 1.0 / sqrt(nrm) : 0.0;
            for (int i = 0; i < N; ++i) SG_L(z, i) *= inv;
        }
        for (int i = 0; i < N; ++i) zt[(long)i * N + k] = SG_L(z, i);
    }
#undef SG_L
}

// Clusters of consecutive eigenvalues of T with gaps below 1e-5 ||T||
// (Gershgorin norm, floored as in the inverse iteration).  Eigenvectors of
// different clusters come out orthogonal to about eps ||T|| / gap <= 2e-11
// without re-orthogonalisation; a wider threshold chains the closely spaced
// Ritz values of large subspaces into long clusters that one thread
// orthogonalises serially.  One workgroup: the norm by a block reduction,
// the compaction by one thread over the eigenvalues in LDS.
__global__ __launch_bounds__(256) void k_clusters(const double* d, const double* e, const double* lam, int N,
                                                  int* cl_start, int* ncl) {
    extern __shared__ double shc[];
    double* sl = shc;                              // N eigenvalues
    __shared__ double red[4];
    const int t = threadIdx.x;
    double tn = 0.0;
    for (int i = t; i < N; i += blockDim.x) {
        tn = fmax(tn, fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < N ? fabs(e[i]) : 0.0));
        sl[i] = lam[i];
    }
    for (int off = 32; off > 0; off >>= 1) tn = fmax(tn, __shfl_xor(tn, off, 64));
    if ((t & 63) == 0) red[t >> 6] = tn;
    __syncthreads();
    if (t != 0) return;
    const double tnorm = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    const double gap = 1e-5 * fmax(tnorm, 1e-100);
    int n = 0;
    cl_start[n++] = 0;
    for (int k = 1; k < N; ++k)
        if (sl[k] - sl[k - 1] > gap) cl_start[n++] = k;
    cl_start[n] = N;
    *ncl = n;
}

// Z <- H_0 H_1 ... H_{N-3} Z^T (input zt = Z^T column-major), one wave per
// output column, the column held in LDS while the reflectors are applied;
// Z is written in column-major order.  LDS: 4 N doubles.
__global__ __launch_bounds__(256) void k_backtransform(const double* A, const double* tau, int N, const double* zt,
                                                       double* Z) {
    extern __shared__ double zs[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = blockIdx.x * 4 + wv;
    if (col >= N) return;
    double* zc = zs + (long)wv * N;
    // every element of the column is owned by one lane throughout (no
    // other lane reads or writes it, so no barrier is needed)
    for (int r = lane; r < N; r += 64) zc[r] = zt[(long)r * N + col];
    for (int i = N - 3; i >= 0; --i) {
        const double ti = tau[i];
        if (ti == 0.0) continue;
        const double* vi = A + (long)i * N;   // v[r] at rows r = i+1.. (v[i+1] = 1)
        const int r0 = ((i + 1) & ~63) + lane;
        double s = 0.0;
        for (int r = r0; r < N; r += 64)
            if (r >= i + 1) s += ((r == i + 1) ? 1.0 : vi[r]) * zc[r];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        s *= ti;
        for (int r = r0; r < N; r += 64)
            if (r >= i + 1) zc[r] -= s * ((r == i + 1) ? 1.0 : vi[r]);
    }
    double* out = Z + (long)col * N;
    for (int r = lane; r < N; r += 64) out[r] = zc[r];
}

// A (destroyed) -> ascending eigenvalues eig and eigenvectors V (columns).
// work: eigh_work_doubles(N) doubles.  N <= kEighMaxN (LDS of the
// tridiagonalisation).
sparc_status dense_eigh_tridiag(sparc_gpu_ctx c, double* A, int N, double* V, double* eig, double* work) {
    double* d = work;
    double* e = d + N;
    double* tau = e + N;
    double* lamw = tau + N;
    double* shift = lamw + N;                // 1 (+7 pad)
    int* cl = (int*)(shift + 8);             // N + 2 ints
    int* ncl_d = cl + N + 1;
    const int nthr = div_up(N, 64) * 64;     // threads of the inverse iteration
    double* zt = shift + 8 + N + 2;          // N^2
    double* stw = zt + (size_t)N * N;        // 5 N nthr
    const int threads = std::min(1024, std::max(64, div_up(N, 64) * 64));
    int slot = prof_begin(c, PK_EIG_TRD);
    if (N >= 3 && N >= c->trd_multi_min) {
        // zt and stw are free until the inverse iteration
        sparc_status st = sytrd_multi(c, A, N, c->trd_tail, d, e, tau, shift, zt);
        if (st != SPARC_OK) return st;
    } else {
        const size_t trd_lds = (3 * (size_t)N + std::max(1024, N + 64)) * sizeof(double);
        k_sytrd<<<1, threads, trd_lds, c->stream>>>(A, N, d, e, tau, shift);
        SG_CHECK_LAUNCH(c);
    }
    prof_end(c, slot);
    slot = prof_begin(c, PK_EIG_BIS);
    k_bisect<<<N, 64, 2 * N * sizeof(double), c->stream>>>(d, e, N, shift, lamw, eig);
    SG_CHECK_LAUNCH(c);
    prof_end(c, slot);
    slot = prof_begin(c, PK_EIG_VEC);
    k_clusters<<<1, 256, N * sizeof(double), c->stream>>>(d, e, lamw, N, cl, ncl_d);
    SG_CHECK_LAUNCH(c);
    {
        // threads per workgroup whose LU factors and vector fit in LDS; with
        // fewer than 3 per workgroup (N above about 800) LDS caps the solves
        // in flight, and the factors in global memory (every solve at once)
        // are faster: N = 1200 3.2 against 4.2 ms, N = 2000 6.1 against 20.5
        const long lds_doubles = (150L * 1024) / 8;
        const int tpw = (int)std::min<long>(64, (lds_doubles - 2L * N) / (6L * N));
        if (tpw >= std::max(1, c->stein_lds_min_tpw)) {
            const size_t lds = (2 * (size_t)N + 6 * (size_t)N * tpw) * sizeof(double);
            k_stein_lds<<<div_up(N, tpw), 64, lds, c->stream>>>(d, e, lamw, N, cl, ncl_d, zt, tpw);
        } else {
            k_stein<<<nthr / 64, 64, 0, c->stream>>>(d, e, lamw, N, cl, ncl_d, zt, stw);
        }
    }
    SG_CHECK_LAUNCH(c);
    if (c->debug) {
        std::vector<int> h(N + 2);
        SG_HIP(c, hipMemcpyAsync(h.data(), cl, (N + 2) * sizeof(int), hipMemcpyDeviceToHost, c->stream));
        SG_HIP(c, hipStreamSynchronize(c->stream));
        const int n = h[N + 1];
        int mx = 0, multi = 0;
        for (int q = 0; q < n; ++q) {
            const int sz = h[q + 1] - h[q];
            mx = std::max(mx, sz);
            multi += sz > 1 ? sz : 0;
        }
        fprintf(stderr, "[sparc_gpu] eigh N=%d clusters %d, largest %d, states in clusters of >1: %d\n", N, n, mx,
                multi);
    }
    prof_end(c, slot);
    slot = prof_begin(c, PK_EIG_BACK);
    k_backtransform<<<div_up(N, 4), 256, 4 * (size_t)N * sizeof(double), c->stream>>>(A, tau, N, zt, V);
    SG_CHECK_LAUNCH(c);
    prof_end(c, slot);
    return SPARC_OK;
}

}  // namespace sg
