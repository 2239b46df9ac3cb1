// FP64 subspace algebra of Rayleigh-Ritz (the N_s x N_s part of CheFSI,
// Sec. 2.1; the paper notes its cubic cost limits scaling, Sec. 4):
// Cholesky of the Gram matrix, inverse of its triangular factor, small
// products, and a parallel cyclic Jacobi eigensolver.
//
// All matrices are N x N, column-major, leading dimension N, in device memory.
#include <algorithm>
#include <cmath>
#include <cstdio>

#include "internal.hpp"

namespace sg {

// Pivots at or below this fraction of their original diagonal entry mean a
// numerically rank-deficient block (about 64 units of rounding).
constexpr double kPivotRtol = 64.0 * 2.220446049250313e-16;

// Blocked Cholesky M = L L^T in place (lower triangle), one workgroup.
// Panels of jb columns are loaded into LDS, factored there column by column
// (left-looking inside the panel), written back, and the trailing lower
// triangle receives one rank-jb update per panel (each element read and
// written once per panel).  flag[0] is set on a non-positive (relative)
// pivot or a non-finite entry.
__global__ __launch_bounds__(1024) void k_cholesky(double* M, int N, int jbmax, int* flag) {
    extern __shared__ double sh[];
    double* dorig = sh;            // N original diagonal entries
    double* P = sh + N;            // panel: (N - j0) rows x jb columns, row-major
    __shared__ int bad;
    __shared__ double piv;
    const int t = threadIdx.x, nt = blockDim.x;
    for (int i = t; i < N; i += nt) dorig[i] = M[i + (long)i * N];
    if (t == 0) bad = 0;
    __syncthreads();
    for (int j0 = 0; j0 < N; j0 += jbmax) {
        const int jb = min(jbmax, N - j0);
        const int nr = N - j0;
        for (int q = t; q < nr * jb; q += nt) {
            const int r = q / jb, p = q - r * jb;
            P[q] = M[(j0 + r) + (long)(j0 + p) * N];
        }
        __syncthreads();
        for (int p = 0; p < jb; ++p) {
            // column p of the panel minus the earlier panel columns
            for (int r = p + t; r < nr; r += nt) {
                double v = P[r * jb + p];
                for (int q = 0; q < p; ++q) v -= P[r * jb + q] * P[p * jb + q];
                P[r * jb + p] = v;
            }
            __syncthreads();
            if (t == 0) {
                const double d = P[p * jb + p];
                if (!(d > kPivotRtol * dorig[j0 + p]) || !isfinite(d)) {
                    bad = 1;
                } else {
                    piv = sqrt(d);
                }
            }
            __syncthreads();
            if (bad) {
                if (t == 0) flag[0] = 1;
                return;
            }
            const double ljj = piv, inv = 1.0 / ljj;
            for (int r = p + t; r < nr; r += nt) P[r * jb + p] = (r == p) ? ljj : P[r * jb + p] * inv;
            __syncthreads();
        }
        for (int q = t; q < nr * jb; q += nt) {
            const int r = q / jb, p = q - r * jb;
            M[(j0 + r) + (long)(j0 + p) * N] = P[q];
        }
        // trailing update of the lower triangle: rows i >= k >= j0 + jb
        const int k0 = j0 + jb;
        const int m = N - k0;
        if (m > 0) {
            const int R = ((m + 63) / 64) * 64;
            const int G = max(1, min(16, nt / R));
            const int TPG = ((nt / G) / 64) * 64;
            const int grp = t / TPG, lr0 = t - grp * TPG;
            if (grp < G) {
                for (int lr = lr0; lr < m; lr += TPG) {
                    const int i = k0 + lr;
                    const double* Pi = P + (i - j0) * jb;
                    int k = k0 + grp;
                    for (; k + 3 * G <= i; k += 4 * G) {
                        double* a0 = M + i + (long)k * N;
                        double x0 = a0[0], x1 = a0[(long)G * N], x2 = a0[(long)2 * G * N], x3 = a0[(long)3 * G * N];
                        const double* P0 = P + (k - j0) * jb;
                        const double* P1 = P0 + G * jb;
                        const double* P2 = P1 + G * jb;
                        const double* P3 = P2 + G * jb;
                        for (int q = 0; q < jb; ++q) {
                            const double pi = Pi[q];
                            x0 -= pi * P0[q];
                            x1 -= pi * P1[q];
                            x2 -= pi * P2[q];
                            x3 -= pi * P3[q];
                        }
                        a0[0] = x0;
                        a0[(long)G * N] = x1;
                        a0[(long)2 * G * N] = x2;
                        a0[(long)3 * G * N] = x3;
                    }
                    for (; k <= i; k += G) {
                        double* a0 = M + i + (long)k * N;
                        double x0 = a0[0];
                        const double* P0 = P + (k - j0) * jb;
                        for (int q = 0; q < jb; ++q) x0 -= Pi[q] * P0[q];
                        a0[0] = x0;
                    }
                }
            }
        }
        __syncthreads();
    }
    // zero the strict upper triangle so that M holds exactly L
    for (long f = t; f < (long)N * N; f += nt) {
        int i = (int)(f % N), k = (int)(f / N);
        if (k > i) M[f] = 0.0;
    }
}

// ---- the same factorisation over many workgroups (large N) ---------------
// Per panel: one workgroup factors it exactly as k_cholesky does, then a
// grid of 64 x 64 tiles applies its rank-jb update to the trailing lower
// triangle.  Each entry receives the same operations in the same order as
// in k_cholesky, so the factor is bitwise the same.

__global__ void k_chol_diag(const double* __restrict__ M, int N, double* __restrict__ dorig) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) dorig[i] = M[i + (long)i * N];
}

// Panel columns j0 .. j0 + jb - 1, rows j0 .. N - 1.  On a bad pivot the
// panel is not written back and flag[0] is set.
__global__ __launch_bounds__(1024) void k_chol_panel(double* M, int N, int j0, int jb,
                                                     const double* __restrict__ dorig, int* flag) {
    extern __shared__ double P[];  // (N - j0) rows x jb columns, row-major
    __shared__ int bad;
    __shared__ double piv;
    const int t = threadIdx.x, nt = blockDim.x;
    const int nr = N - j0;
    if (t == 0) bad = 0;
    for (int q = t; q < nr * jb; q += nt) {
        const int r = q / jb, p = q - r * jb;
        P[q] = M[(j0 + r) + (long)(j0 + p) * N];
    }
    __syncthreads();
    for (int p = 0; p < jb; ++p) {
        for (int r = p + t; r < nr; r += nt) {
            double v = P[r * jb + p];
            for (int q = 0; q < p; ++q) v -= P[r * jb + q] * P[p * jb + q];
            P[r * jb + p] = v;
        }
        __syncthreads();
        if (t == 0) {
            const double d = P[p * jb + p];
            if (!(d > kPivotRtol * dorig[j0 + p]) || !isfinite(d)) {
                bad = 1;
            } else {
                piv = sqrt(d);
            }
        }
        __syncthreads();
        if (bad) {
            if (t == 0) flag[0] = 1;
            return;
        }
        const double ljj = piv, inv = 1.0 / ljj;
        for (int r = p + t; r < nr; r += nt) P[r * jb + p] = (r == p) ? ljj : P[r * jb + p] * inv;
        __syncthreads();
    }
    for (int q = t; q < nr * jb; q += nt) {
        const int r = q / jb, p = q - r * jb;
        M[(j0 + r) + (long)(j0 + p) * N] = P[q];
    }
}

constexpr int kCholT = 64;  // trailing-update tile edge

// A[i][k] -= sum_q L[i][j0+q] L[k][j0+q] for k0 <= k <= i < N, tile
// (blockIdx.x, blockIdx.y) = (row block, column block); jb <= 16.
__global__ __launch_bounds__(256) void k_chol_update(double* M, int N, int k0, int j0, int jb) {
    const int bi = blockIdx.x, bk = blockIdx.y;
    if (bi < bk) return;
    __shared__ double Li[kCholT][16], Lk[kCholT][16];
    const int t = threadIdx.x;
    const int i0 = k0 + bi * kCholT, c0 = k0 + bk * kCholT;
    for (int q = t; q < kCholT * jb; q += blockDim.x) {
        const int r = q % kCholT, p = q / kCholT;
        const int gi = i0 + r, gk = c0 + r;
        Li[r][p] = gi < N ? M[gi + (long)(j0 + p) * N] : 0.0;
        Lk[r][p] = gk < N ? M[gk + (long)(j0 + p) * N] : 0.0;
    }
    __syncthreads();
    const int r = t & (kCholT - 1);
    const int i = i0 + r;
    if (i >= N) return;
    for (int kc = t >> 6; kc < kCholT; kc += blockDim.x / kCholT) {
        const int k = c0 + kc;
        if (k > i) break;
        double* a = M + i + (long)k * N;
        double x = *a;
        for (int q = 0; q < jb; ++q) x -= Li[r][q] * Lk[kc][q];
        *a = x;
    }
}

__global__ void k_zero_upper(double* M, int N) {
    const long f = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= (long)N * N) return;
    const int i = (int)(f % N), k = (int)(f / N);
    if (k > i) M[f] = 0.0;
}

sparc_status dense_cholesky(sparc_gpu_ctx c, double* M, int N, int* flag) {
    const int slot = prof_begin(c, PK_CHOL);
    // panel width: the panel (N x jb) and the original diagonal fit in LDS
    const int jb = std::max(1, std::min(16, (int)((120 * 1024) / (8 * (size_t)N))));
    if (N >= c->chol_multi_min) {
        if (!c->chol_dorig) SG_HIP(c, hipMalloc((void**)&c->chol_dorig, kEighMaxN * sizeof(double)));
        if (N > kEighMaxN) return set_err(c, SPARC_ERR_ARG, "cholesky: N above the subspace limit");
        k_chol_diag<<<div_up(N, 256), 256, 0, c->stream>>>(M, N, c->chol_dorig);
        for (int j0 = 0; j0 < N; j0 += jb) {
            const int w = std::min(jb, N - j0);
            k_chol_panel<<<1, 1024, (size_t)(N - j0) * w * sizeof(double), c->stream>>>(M, N, j0, w, c->chol_dorig,
                                                                                      flag);
            const int k0 = j0 + w, m = N - k0;
            if (m > 0) {
                const int nb = div_up(m, kCholT);
                k_chol_update<<<dim3(nb, nb), 256, 0, c->stream>>>(M, N, k0, j0, w);
            }
        }
        k_zero_upper<<<div_up((long)N * N, 256L), 256, 0, c->stream>>>(M, N);
        SG_CHECK_LAUNCH(c);
        prof_end(c, slot);
        return SPARC_OK;
    }
    const size_t lds = ((size_t)N + (size_t)N * jb) * sizeof(double);
    k_cholesky<<<1, 1024, lds, c->stream>>>(M, N, jb, flag);
    SG_CHECK_LAUNCH(c);
    prof_end(c, slot);
    return SPARC_OK;
}

__global__ void k_transpose(const double* A, double* B, int N) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)N * N) return;
    int i = (int)(e % N), j = (int)(e / N);
    B[j + (long)i * N] = A[e];
}

// Column j of L^-1 by forward substitution, one wave per column; Lt = L^T
// (so that row i of L is contiguous).
__global__ __launch_bounds__(64) void k_tri_inv_col(const double* __restrict__ Lt, double* __restrict__ Linv, int N) {
    extern __shared__ double xs[];
    const int j = blockIdx.x, lane = threadIdx.x;
    for (int i = lane; i < N; i += 64) xs[i] = 0.0;
    __syncthreads();
    if (lane == 0) xs[j] = 1.0 / Lt[j + (long)j * N];
    __syncthreads();
    for (int i = j + 1; i < N; ++i) {
        const double* li = Lt + (long)i * N;  // L[i][k] = Lt[k + i N]
        double s = 0.0;
        for (int k = j + lane; k < i; k += 64) s += li[k] * xs[k];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        s = __shfl(s, 0, 64);
        if (lane == 0) xs[i] = -s / li[i];
        __syncthreads();
    }
    for (int i = lane; i < N; i += 64) Linv[i + (long)j * N] = xs[i];
}

sparc_status dense_tri_inverse_lower(sparc_gpu_ctx c, const double* L, double* Linv, int N) {
    // Linv doubles as scratch for L^T first
    double* Lt = c->small + 8 * (size_t)N * N;
    const int slot = prof_begin(c, PK_TRINV);
    k_transpose<<<div_up((long)N * N, 256), 256, 0, c->stream>>>(L, Lt, N);
    SG_CHECK_LAUNCH(c);
    k_tri_inv_col<<<N, 64, N * sizeof(double), c->stream>>>(Lt, Linv, N);
    SG_CHECK_LAUNCH(c);
    prof_end(c, slot);
    return SPARC_OK;
}

// C = op(A) op(B), 16x16 tiles through LDS.
__global__ __launch_bounds__(256) void k_small_gemm(int N, const double* __restrict__ A, bool ta,
                                                    const double* __restrict__ B, bool tb, double* __restrict__ C) {
    __shared__ double sA[16][17], sB[16][17];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i = blockIdx.x * 16 + tx;  // row of C
    const int j = blockIdx.y * 16 + ty;  // column of C
    double acc = 0.0;
    for (int k0 = 0; k0 < N; k0 += 16) {
        // sA[tx][ty] = op(A)[i][k0 + ty]; sB[tx][ty] = op(B)[k0 + tx][j]
        int k = k0 + ty;
        double va = 0.0;
        if (i < N && k < N) va = ta ? A[k + (long)i * N] : A[i + (long)k * N];
        int kb = k0 + tx;
        double vb = 0.0;
        if (j < N && kb < N) vb = tb ? B[j + (long)kb * N] : B[kb + (long)j * N];
        sA[tx][ty] = va;
        sB[tx][ty] = vb;
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) acc += sA[tx][kk] * sB[kk][ty];
        __syncthreads();
    }
    if (i < N && j < N) C[i + (long)j * N] = acc;
}

sparc_status dense_gemm(sparc_gpu_ctx c, char ta, char tb, int N, const double* A, const double* B, double* C) {
    dim3 grid(div_up(N, 16), div_up(N, 16));
    const int slot = prof_begin(c, PK_SMALL);
    k_small_gemm<<<grid, 256, 0, c->stream>>>(N, A, ta == 'T', B, tb == 'T', C);
    SG_CHECK_LAUNCH(c);
    prof_end(c, slot);
    return SPARC_OK;
}

__global__ void k_symmetrize(double* A, int N) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)N * N) return;
    int i = (int)(e % N), j = (int)(e / N);
    if (i < j) {
        double v = 0.5 * (A[i + (long)j * N] + A[j + (long)i * N]);
        A[i + (long)j * N] = v;
        A[j + (long)i * N] = v;
    }
}

sparc_status dense_symmetrize(sparc_gpu_ctx c, double* A, int N) {
    k_symmetrize<<<div_up((long)N * N, 256), 256, 0, c->stream>>>(A, N);
    SG_CHECK_LAUNCH(c);
    return SPARC_OK;
}

// ---------------------------------------------------------------- Jacobi

// Round-robin pairing of P (even) players over rounds r = 0..P-2: player
// P-1 meets r; any other i meets (2r - i) mod (P-1).
__device__ inline int partner(int i, int r, int P) {
    if (i == P - 1) return r;
    if (i == r) return P - 1;
    int q = (2 * r - i) % (P - 1);
    return q < 0 ? q + (P - 1) : q;
}

// Rotation (c, g) of index i in round r: column i of J has J_ii = c and
// J_{p(i), i} = g; for the pair lo < hi, t = sgn(z)/(|z| + sqrt(1 + z^2)),
// z = (a_hh - a_ll) / (2 a_lh), c = 1/sqrt(1 + t^2), s = t c, g = -s at lo
// and +s at hi; this zeroes a_lh.
__device__ inline void rotation(const double* A, int N, int i, int p, double& cc, double& g) {
    cc = 1.0;
    g = 0.0;
    if (p >= N || p == i) return;
    int lo = min(i, p), hi = max(i, p);
    double all = A[lo + (long)lo * N], ahh = A[hi + (long)hi * N], alh = A[lo + (long)hi * N];
    if (alh == 0.0) return;
    double z = (ahh - all) / (2.0 * alh);
    double t = (z >= 0.0 ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z));
    double cs = 1.0 / sqrt(1.0 + t * t);
    double s = t * cs;
    cc = cs;
    g = (i == lo) ? -s : s;
}

// A' = J^T A J and V' = V J for one round of disjoint rotations.
__global__ __launch_bounds__(256) void k_jacobi_round(const double* __restrict__ A, double* __restrict__ An,
                                                      const double* __restrict__ V, double* __restrict__ Vn, int N,
                                                      int P, int r) {
    __shared__ double ci[16], gi[16], cj[16], gj[16];
    __shared__ int pi[16], pj[16];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i0 = blockIdx.x * 16, j0 = blockIdx.y * 16;
    if (threadIdx.x < 16) {
        int i = i0 + threadIdx.x;
        if (i < N) {
            int p = partner(i, r, P);
            double cc, g;
            rotation(A, N, i, p, cc, g);
            ci[threadIdx.x] = cc;
            gi[threadIdx.x] = g;
            pi[threadIdx.x] = p < N ? p : i;
        }
    } else if (threadIdx.x < 32) {
        int j = j0 + threadIdx.x - 16;
        if (j < N) {
            int p = partner(j, r, P);
            double cc, g;
            rotation(A, N, j, p, cc, g);
            cj[threadIdx.x - 16] = cc;
            gj[threadIdx.x - 16] = g;
            pj[threadIdx.x - 16] = p < N ? p : j;
        }
    }
    __syncthreads();
    const int i = i0 + tx, j = j0 + ty;
    if (i >= N || j >= N) return;
    const double c_i = ci[tx], g_i = gi[tx], c_j = cj[ty], g_j = gj[ty];
    const int p_i = pi[tx], p_j = pj[ty];
    double v = c_i * c_j * A[i + (long)j * N] + c_i * g_j * A[i + (long)p_j * N] +
               g_i * c_j * A[p_i + (long)j * N] + g_i * g_j * A[p_i + (long)p_j * N];
    An[i + (long)j * N] = v;
    // V' = V J: row i of V, column j
    Vn[i + (long)j * N] = V[i + (long)j * N] * c_j + V[i + (long)p_j * N] * g_j;
}

__global__ void k_identity(double* V, int N) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)N * N) return;
    V[e] = ((e % N) == (e / N)) ? 1.0 : 0.0;
}

// out[0] = sum_{i != j} A_ij^2, out[1] = sum A_ij^2 (one block, fixed order)
__global__ void k_offnorm(const double* A, int N, double* out) {
    __shared__ double s0[1024], s1[1024];
    double a = 0.0, b = 0.0;
    for (long e = threadIdx.x; e < (long)N * N; e += blockDim.x) {
        double v = A[e] * A[e];
        b += v;
        if ((e % N) != (e / N)) a += v;
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = b;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            s0[threadIdx.x] += s0[threadIdx.x + s];
            s1[threadIdx.x] += s1[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s0[0];
        out[1] = s1[0];
    }
}

// Ascending order of the diagonal (ties by index) and the matching columns.
__global__ void k_sort_eig(const double* A, const double* V, int N, double* eig, double* Vs) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double di = A[i + (long)i * N];
    int rank = 0;
    for (int j = 0; j < N; ++j) {
        double dj = A[j + (long)j * N];
        if (dj < di || (dj == di && j < i)) ++rank;
    }
    eig[rank] = di;
    for (int k = 0; k < N; ++k) Vs[k + (long)rank * N] = V[k + (long)i * N];
}

__global__ void k_copy2(const double* __restrict__ a2, double* __restrict__ a, const double* __restrict__ v2,
                        double* __restrict__ v, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        a[i] = a2[i];
        v[i] = v2[i];
    }
}

// One Jacobi sweep (P-1 rounds ping-ponging between (A, V) and (A2, V2),
// ending in (A, V)) as a HIP graph, captured once per matrix size and
// buffer set on a private stream and replayed on the context's stream; the
// sweep is hundreds of tiny launches, so this removes their launch cost.
static sparc_status jacobi_sweep(sparc_gpu_ctx c, double* A, double* A2, double* V, double* V2, int N, int P) {
    if (!c->jac_exec || c->jac_N != N || c->jac_A != A || c->jac_A2 != A2 || c->jac_V != V || c->jac_V2 != V2) {
        if (c->jac_exec) {
            hipGraphExecDestroy(c->jac_exec);
            c->jac_exec = nullptr;
        }
        if (!c->cap_stream) SG_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        SG_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        dim3 grid(div_up(N, 16), div_up(N, 16));
        double *Ac = A, *An = A2, *Vc = V, *Vn = V2;
        for (int r = 0; r < P - 1; ++r) {
            k_jacobi_round<<<grid, 256, 0, c->cap_stream>>>(Ac, An, Vc, Vn, N, P, r);
            std::swap(Ac, An);
            std::swap(Vc, Vn);
        }
        if (Ac != A) k_copy2<<<div_up((long)N * N, 256), 256, 0, c->cap_stream>>>(A2, A, V2, V, (long)N * N);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
        if (e != hipSuccess) return hip_err(c, e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&c->jac_exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_err(c, e, "hipGraphInstantiate");
        c->jac_N = N;
        c->jac_A = A;
        c->jac_A2 = A2;
        c->jac_V = V;
        c->jac_V2 = V2;
    }
    SG_HIP(c, hipGraphLaunch(c->jac_exec, c->stream));
    return SPARC_OK;
}

// A (destroyed), V: N x N; eig: N; work: 2 N^2 doubles.
sparc_status dense_eigh(sparc_gpu_ctx c, double* A, int N, double* V, double* eig, double* work) {
    const int P = N + (N & 1);
    double* A2 = work;
    double* V2 = work + (size_t)N * N;
    k_identity<<<div_up((long)N * N, 256), 256, 0, c->stream>>>(V, N);
    SG_CHECK_LAUNCH(c);
    double* Acur = A;
    double* Anext = A2;
    double* Vcur = V;
    double* Vnext = V2;
    const int max_sweeps = 40;
    bool converged = false;
    // Off-diagonal mass at the rounding floor of the rotations (each element
    // is recomputed with O(eps ||A||) error), so ask for (4 N eps)^2 ||A||_F^2.
    const double ne = 4.0 * N * 2.220446049250313e-16;
    const double tol = std::max(ne * ne, 1e-30);
    double prev_off = -1.0;
    dim3 grid(div_up(N, 16), div_up(N, 16));
    double* d_norm = c->scal + S_EIG;
    for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
        k_offnorm<<<1, 1024, 0, c->stream>>>(Acur, N, d_norm);
        SG_CHECK_LAUNCH(c);
        double h[2];
        SG_HIP(c, hipMemcpyAsync(h, d_norm, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        SG_HIP(c, hipStreamSynchronize(c->stream));
        if (!std::isfinite(h[0]) || !std::isfinite(h[1])) return set_err(c, SPARC_ERR_NONFINITE, "eigh: non-finite");
        if (c->debug) fprintf(stderr, "[sparc_gpu] eigh N=%d sweep %d off^2/norm^2 %.3e\n", N, sweep, h[0] / h[1]);
        if (h[0] <= tol * h[1] || h[1] == 0.0) {
            converged = true;
            break;
        }
        // stagnation at the rounding floor also counts as converged
        if (prev_off >= 0.0 && h[0] <= 1e-20 * h[1] && h[0] >= 0.25 * prev_off) {
            converged = true;
            break;
        }
        prev_off = h[0];
        sparc_status st = jacobi_sweep(c, Acur, Anext, Vcur, Vnext, N, P);
        if (st != SPARC_OK) return st;
    }
    if (!converged) return set_err(c, SPARC_ERR_EIG, "Jacobi eigensolver did not converge");
    // sorted result into eig and V (V may currently live in work)
    double* Vs = (Vcur == V) ? V2 : V;
    k_sort_eig<<<div_up(N, 128), 128, 0, c->stream>>>(Acur, Vcur, N, eig, Vs);
    SG_CHECK_LAUNCH(c);
    if (Vs != V) SG_HIP(c, hipMemcpyAsync(V, Vs, (size_t)N * N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return SPARC_OK;
}

// ---------------------------------------------------------------- Rayleigh-Ritz

template <typename T>
__global__ void k_copy_cols(const T* __restrict__ src, T* __restrict__ dst, long nd, int ncol, long ld) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    if (i < nd && j < ncol) dst[i + (long)j * ld] = src[i + (long)j * ld];
}

// X <- Y R^-1 Q with dV Y^T Y = R^T R (R = L^T) and
// R^-T (dV Y^T H Y) R^-1 = Q diag(eig) Q^T, for columns of `rows` values
// (N_d, or 2 N_d for Bloch columns) and the operator applied by applyH(Y, W).
// Workspace: c->work (one block) and c->small (>= 12 N^2 doubles).
template <typename T, typename ApplyH>
static sparc_status rr_core(sparc_gpu_ctx c, T* X, int N, long ldx, double* d_eig, bool check, long rows,
                            ApplyH&& applyH) {
    sparc_status st;
    const size_t blk = ((size_t)(N - 1) * ldx + rows) * sizeof(T);
    if ((st = ensure_work(c, blk)) != SPARC_OK) return st;
    if ((st = ensure_small(c, 9 * (size_t)N * N + eigh_work_doubles(N))) != SPARC_OK) return st;
    T* W = (T*)c->work;
    const size_t NN = (size_t)N * N;
    double* M = c->small;           // Gram, then L
    double* Linv = M + NN;
    double* K = M + 2 * NN;         // dV Y^T H Y
    double* T1 = M + 3 * NN;
    double* Hs = M + 4 * NN;
    double* Vq = M + 5 * NN;
    double* Rot = M + 6 * NN;
    double* ework = M + 9 * NN;     // eigensolver workspace; Lt lives at 8 NN
    // the public call starts from a clear flag; inside an SCF step the flag
    // was cleared at the step's start and must survive every pass
    if (check) SG_HIP(c, hipMemsetAsync(c->flags + F_NOT_SPD, 0, sizeof(int), c->stream));
    if ((st = gemm_tn<T>(c, N, N, rows, X, ldx, X, ldx, c->dV, M, N, true)) != SPARC_OK) return st;
    if ((st = dense_cholesky(c, M, N, c->flags + F_NOT_SPD)) != SPARC_OK) return st;
    if (check) {
        int f = 0;
        SG_HIP(c, hipMemcpyAsync(&f, c->flags + F_NOT_SPD, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        SG_HIP(c, hipStreamSynchronize(c->stream));
        if (f) return set_err(c, SPARC_ERR_NOT_SPD, "Gram matrix of the block is not positive definite");
    }
    if ((st = dense_tri_inverse_lower(c, M, Linv, N)) != SPARC_OK) return st;
    // H Y into W
    if ((st = applyH(X, W)) != SPARC_OK) return st;
    // dV Y^T (H Y) is symmetric (H is): its upper tiles are computed and mirrored
    if ((st = gemm_tn<T>(c, N, N, rows, X, ldx, W, ldx, c->dV, K, N, true)) != SPARC_OK) return st;
    if ((st = dense_gemm(c, 'N', 'N', N, Linv, K, T1)) != SPARC_OK) return st;
    if ((st = dense_gemm(c, 'N', 'T', N, T1, Linv, Hs)) != SPARC_OK) return st;
    if ((st = dense_symmetrize(c, Hs, N)) != SPARC_OK) return st;
    {
        const int slot = prof_begin(c, PK_EIG);
        st = c->eig_jacobi ? dense_eigh(c, Hs, N, Vq, d_eig, ework) : dense_eigh_tridiag(c, Hs, N, Vq, d_eig, ework);
        prof_end(c, slot);
        if (st != SPARC_OK) return st;
    }
    if ((st = dense_gemm(c, 'T', 'N', N, Linv, Vq, Rot)) != SPARC_OK) return st;
    if ((st = gemm_nn<T>(c, rows, N, N, X, ldx, Rot, N, W, ldx)) != SPARC_OK) return st;
    dim3 grid(div_up(rows, 256), N);
    const int slot = prof_begin(c, PK_COPY);
    k_copy_cols<T><<<grid, 256, 0, c->stream>>>(W, X, rows, N, ldx);
    SG_CHECK_LAUNCH(c);
    prof_end(c, slot);
    return SPARC_OK;
}

template <typename T>
sparc_status rayleigh_ritz_impl(sparc_gpu_ctx c, T* X, int N, long ldx, double* d_eig, bool check) {
    return rr_core<T>(c, X, N, ldx, d_eig, check, c->nd, [&](T* Y, T* W) -> sparc_status {
        sparc_status st = launch_projection<T>(c, Y, N, ldx);
        if (st != SPARC_OK) return st;
        return launch_hsweep<T>(c, Y, W, nullptr, N, ldx, 0, 0);
    });
}

// Bloch columns at the context's k: the real embedding of the Hermitian H_k.
template <typename T>
sparc_status rayleigh_ritz_k_impl(sparc_gpu_ctx c, T* X, int N, long ldx, double* d_eig, bool check) {
    return rr_core<T>(c, X, N, ldx, d_eig, check, 2 * c->nd,
                      [&](T* Y, T* W) -> sparc_status { return bloch_apply_impl<T>(c, Y, W, N, ldx); });
}

template sparc_status rayleigh_ritz_k_impl<double>(sparc_gpu_ctx, double*, int, long, double*, bool);
template sparc_status rayleigh_ritz_k_impl<float>(sparc_gpu_ctx, float*, int, long, double*, bool);

template sparc_status rayleigh_ritz_impl<double>(sparc_gpu_ctx, double*, int, long, double*, bool);
template sparc_status rayleigh_ritz_impl<float>(sparc_gpu_ctx, float*, int, long, double*, bool);

}  // namespace sg

using namespace sg;

extern "C" sparc_status sparc_gpu_subspace_eigh(sparc_gpu_ctx c, double* d_A, int n, double* d_V, double* d_eig) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    if (!d_A || !d_V || !d_eig) return set_err(c, SPARC_ERR_ARG, "subspace_eigh: null pointer");
    if (n < 1 || n > kEighMaxN) return set_err(c, SPARC_ERR_ARG, "subspace_eigh: n out of range");
    sparc_status st = ensure_small(c, eigh_work_doubles(n));
    if (st != SPARC_OK) return st;
    double* work = c->small;
    st = c->eig_jacobi ? dense_eigh(c, d_A, n, d_V, d_eig, work) : dense_eigh_tridiag(c, d_A, n, d_V, d_eig, work);
    if (st != SPARC_OK) return st;
    SG_HIP(c, hipStreamSynchronize(c->stream));
    return SPARC_OK;
}

extern "C" sparc_status sparc_gpu_rayleigh_ritz(sparc_gpu_ctx c, sparc_prec prec, void* d_X, int ncol, long ldx,
                                                double* d_eig) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    if (prec != SPARC_FP64 && prec != SPARC_FP32) return set_err(c, SPARC_ERR_ARG, "rayleigh_ritz: bad precision");
    if (!d_X || !d_eig) return set_err(c, SPARC_ERR_ARG, "rayleigh_ritz: null pointer");
    if (ncol < 1 || ncol > c->n_states) return set_err(c, SPARC_ERR_ARG, "rayleigh_ritz: ncol out of range");
    if (ldx < c->nd) return set_err(c, SPARC_ERR_ARG, "rayleigh_ritz: ldx < N_d");
    sparc_status st;
    if (prec == SPARC_FP64)
        st = rayleigh_ritz_impl<double>(c, (double*)d_X, ncol, ldx, d_eig, true);
    else
        st = rayleigh_ritz_impl<float>(c, (float*)d_X, ncol, ldx, d_eig, true);
    if (st != SPARC_OK) return st;
    SG_HIP(c, hipStreamSynchronize(c->stream));
    return SPARC_OK;
}
