// Dense subspace products of Rayleigh-Ritz on MFMA (the Gram matrix
// dV Y^T Y, the projected Hamiltonian dV Y^T (H Y) and the rotation Y T).
//
// gemm_tn: C = alpha A^T B for tall-skinny A (K x M), B (K x N), K = N_d.
//   Deterministic split-K: each workgroup reduces one K-chunk of one 64x64
//   tile on MFMA (FP64 MFMA for double; FP32 MFMA with FP32 accumulation
//   inside the chunk for float) and writes a double partial; a second kernel
//   sums the partials in a fixed order in double.
// gemm_nn: Out = A Bm with A tall (K x M), Bm small (M x N, double, rounded
//   to the block precision).
//
// MFMA 16x16x4 operand layout (one wave): lane l supplies A[i = l%16][k = l/16]
// and B[k = l/16][j = l%16].  Accumulator register r of lane l holds
// C[i][j = l%16] with i = 4*(l/16) + r for the f32 instruction and
// i = l/16 + 4*r for the f64 one (both measured on gfx950).
#include "internal.hpp"

namespace sg {

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    typedef double acc_t __attribute__((ext_vector_type(4)));
    static __device__ inline acc_t run(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mfma<float> {
    typedef float acc_t __attribute__((ext_vector_type(4)));
    static __device__ inline acc_t run(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Workgroup = 2 x 2 waves; a wave owns (16 MT) x (16 NT) outputs as MT x NT
// MFMA 16x16 tiles, so a workgroup tile is (32 MT) x (32 NT).  Operands pass
// through LDS in stages of BK = 16 along the contraction, double-buffered
// (the next stage's global loads are issued before the current stage's MFMAs
// and written to the other buffer after them: one barrier per stage).
constexpr int BK = 16;
constexpr int PAD = 2;

// One stage of MFMAs from LDS: sa[k][row], sb[k][col].
template <typename T, int MT, int NT>
__device__ __forceinline__ void mfma_stage(const T* sa, int lda_s, const T* sb, int ldb_s, int wr0, int wc0, int lane,
                                           typename Mfma<T>::acc_t (&acc)[MT][NT]) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
        T av[MT], bv[NT];
        const int kr = kk + (lane >> 4), li = lane & 15;
#pragma unroll
        for (int i = 0; i < MT; ++i) av[i] = sa[kr * lda_s + wr0 + 16 * i + li];
#pragma unroll
        for (int j = 0; j < NT; ++j) bv[j] = sb[kr * ldb_s + wc0 + 16 * j + li];
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int j = 0; j < NT; ++j) acc[i][j] = Mfma<T>::run(av[i], bv[j], acc[i][j]);
    }
}

// Partial[split][n][m] = sum_{k in chunk} A[k, m] B[k, n] for one tile of
// (32 MT) x (32 NT) outputs.  A, B are K x M / K x N column-major.
//
// One workgroup per (active tile, split); only the upper tiles tn >= tm are
// active when `symmetric`.  Hardware dispatches block b to XCD b % 8.  When
// nsplit is a multiple of 8, every tile of one split runs on one XCD, and
// its tiles are dispatched together, so that the panels of that K-chunk,
// which a tile row or column shares, come from HBM about once and then from
// the XCD's L2 (wholly so while one split's tiles fit the XCD's workgroup
// slots: up to 64 tiles of 128 x 128).
template <typename T, int MT, int NT>
__global__ __launch_bounds__(256) void k_gemm_tn_split(int M, int N, long K, long kchunk, const T* __restrict__ A,
                                                       long lda, const T* __restrict__ B, long ldb,
                                                       double* __restrict__ part, int tiles_m, bool symmetric,
                                                       int active, int nsplit) {
    using acc_t = typename Mfma<T>::acc_t;
    constexpr int TM = 32 * MT, TN = 32 * NT;
    constexpr int LA = TM + PAD, LB = TN + PAD;
    __shared__ T sA[2][BK * LA];
    __shared__ T sB[2][BK * LB];
    const int bid = blockIdx.x;
    int split, tidx;
    if (nsplit % 8 == 0) {
        const int slot = bid / 8;
        split = bid % 8 + 8 * (slot / active);
        tidx = slot % active;
    } else {
        split = bid / active;
        tidx = bid % active;
    }
    int tm, tn;
    if (symmetric) {
        // tidx-th upper tile, column by column: (0,0), (0,1), (1,1), (0,2), ...
        tn = 0;
        while ((tn + 1) * (tn + 2) / 2 <= tidx) ++tn;
        tm = tidx - tn * (tn + 1) / 2;
    } else {
        tm = tidx % tiles_m;
        tn = tidx / tiles_m;
    }
    const long k0 = (long)split * kchunk;
    const long k1 = min(K, k0 + kchunk);
    const int m0 = tm * TM, n0 = tn * TN;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wr0 = (wv & 1) * 16 * MT, wc0 = (wv >> 1) * 16 * NT;
    acc_t acc[MT][NT];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
    // loader: thread t reads k = 2 (t % 8) + {0, 1} of columns t / 8 + 32 p
    const int lk = 2 * (t & 7), lc = t >> 3;
    T ra[MT][2], rb[NT][2];
    auto load = [&](long kb) {
#pragma unroll
        for (int p = 0; p < MT; ++p) {
            const int m = m0 + lc + 32 * p;
            const T* q = A + (long)(m < M ? m : 0) * lda;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const long k = kb + lk + u;
                ra[p][u] = (m < M && k < k1) ? q[k] : (T)0;
            }
        }
#pragma unroll
        for (int p = 0; p < NT; ++p) {
            const int n = n0 + lc + 32 * p;
            const T* q = B + (long)(n < N ? n : 0) * ldb;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const long k = kb + lk + u;
                rb[p][u] = (n < N && k < k1) ? q[k] : (T)0;
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int p = 0; p < MT; ++p)
#pragma unroll
            for (int u = 0; u < 2; ++u) sA[buf][(lk + u) * LA + lc + 32 * p] = ra[p][u];
#pragma unroll
        for (int p = 0; p < NT; ++p)
#pragma unroll
            for (int u = 0; u < 2; ++u) sB[buf][(lk + u) * LB + lc + 32 * p] = rb[p][u];
    };
    const long nst = (k1 - k0 + BK - 1) / BK;
    load(k0);
    store(0);
    __syncthreads();
    for (long s = 0; s < nst; ++s) {
        const int buf = (int)(s & 1);
        if (s + 1 < nst) load(k0 + (s + 1) * BK);
        mfma_stage<T, MT, NT>(sA[buf], LA, sB[buf], LB, wr0, wc0, lane, acc);
        if (s + 1 < nst) store(buf ^ 1);
        __syncthreads();
    }
    double* P = part + (long)split * M * N;
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wr0 + 16 * i + Mfma<T>::row(lane, r);
                const int n = n0 + wc0 + 16 * j + (lane & 15);
                if (m < M && n < N) P[m + (long)n * M] = (double)acc[i][j][r];
            }
}

// C = alpha * sum over splits; with `symmetric` only tiles tn >= tm were
// computed and the lower ones are mirrored.
__global__ void k_gemm_reduce(int M, int N, int nsplit, const double* __restrict__ part, double alpha,
                              double* __restrict__ C, int ldc, bool symmetric, int tile) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)M * N) return;
    int m = (int)(e % M), n = (int)(e / M);
    int sm = m, sn = n;
    if (symmetric && (n / tile) < (m / tile)) {
        sm = n;
        sn = m;
    }
    double s = 0.0;
    for (int k = 0; k < nsplit; ++k) s += part[(long)k * M * N + sm + (long)sn * M];
    C[m + (long)n * ldc] = alpha * s;
}

template <typename T, int MT>
static sparc_status gemm_tn_launch(sparc_gpu_ctx c, int M, int N, long K, const T* A, long lda, const T* B, long ldb,
                                   double alpha, double* C, int ldc, bool symmetric) {
    constexpr int TT = 32 * MT;
    const int tiles_m = div_up(M, TT), tiles_n = div_up(N, TT);
    const int tiles = tiles_m * tiles_n;
    const int active = symmetric ? tiles_m * (tiles_m + 1) / 2 : tiles;
    // about two workgroups per CU, in a multiple of 8 splits (one XCD per
    // split at a time), chunks of >= 1024 rows
    const long want = std::max<long>(1, 512 / active);
    int nsplit = 8 * (int)std::max<long>(1, (want + 4) / 8);
    if ((long)nsplit * 1024 > K) nsplit = (int)std::max<long>(1, K / 1024);
    long kchunk = (K + nsplit - 1) / nsplit;
    kchunk = (kchunk + BK - 1) / BK * BK;
    sparc_status st = ensure_gemm_part(c, (size_t)nsplit * M * N);
    if (st != SPARC_OK) return st;
    const long nblocks = (long)active * nsplit;
    if (nblocks > 0x7fffffffL) return set_err(c, SPARC_ERR_ARG, "gemm_tn: too many blocks");
    const int slot = prof_begin(c, PK_GEMM_TN);
    k_gemm_tn_split<T, MT, MT><<<dim3((unsigned)nblocks), 256, 0, c->stream>>>(
        M, N, K, kchunk, A, lda, B, ldb, c->gemm_part, tiles_m, symmetric, active, nsplit);
    SG_CHECK_LAUNCH(c);
    prof_end(c, slot);
    k_gemm_reduce<<<div_up((long)M * N, 256), 256, 0, c->stream>>>(M, N, nsplit, c->gemm_part, alpha, C, ldc,
                                                                   symmetric, TT);
    SG_CHECK_LAUNCH(c);
    return SPARC_OK;
}

template <typename T>
sparc_status gemm_tn(sparc_gpu_ctx c, int M, int N, long K, const T* A, long lda, const T* B, long ldb,
                     double alpha, double* C, int ldc, bool symmetric) {
    if (symmetric && M != N) return set_err(c, SPARC_ERR_ARG, "gemm_tn: symmetric needs M == N");
    const int mx = std::max(M, N);
    if (mx <= 32) return gemm_tn_launch<T, 1>(c, M, N, K, A, lda, B, ldb, alpha, C, ldc, symmetric);
    if (mx <= 64) return gemm_tn_launch<T, 2>(c, M, N, K, A, lda, B, ldb, alpha, C, ldc, symmetric);
    // 160-wide tiles (one wave per SIMD) or 128-wide (two per SIMD): 160 up
    // to two tiles per edge (N <= 320, where 128 would need three), 128
    // above, where the extra tiles keep more workgroups busy (measured at
    // N = 520 and 1200); override SPARC_GPU_GEMM_TILE = 128 | 160
    const int tile = c->gemm_tile > 0 ? c->gemm_tile : (mx <= 320 ? 160 : 128);
    if (tile == 128) return gemm_tn_launch<T, 4>(c, M, N, K, A, lda, B, ldb, alpha, C, ldc, symmetric);
    return gemm_tn_launch<T, 5>(c, M, N, K, A, lda, B, ldb, alpha, C, ldc, symmetric);
}

// Out (rows x N) = A (rows x M) Bm (M x N); a workgroup owns 32 MT rows and
// 32 NT columns.  Bm is double, rounded to T when staged.
template <typename T, int MT, int NT>
__global__ __launch_bounds__(256) void k_gemm_nn(long K, int N, int M, const T* __restrict__ A, long lda,
                                                 const double* __restrict__ Bm, int ldb, T* __restrict__ Out,
                                                 long ldo) {
    using acc_t = typename Mfma<T>::acc_t;
    constexpr int TM = 32 * MT, TN = 32 * NT;
    constexpr int LA = TM + PAD, LB = TN + PAD;
    __shared__ T sA[2][BK * LA];
    __shared__ T sB[2][BK * LB];
    const long r0 = (long)blockIdx.x * TM;
    const int n0 = blockIdx.y * TN;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wr0 = (wv & 1) * 16 * MT, wc0 = (wv >> 1) * 16 * NT;
    acc_t acc[MT][NT];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
    // A loader: rows t % TM, k = t / TM + (256 / TM) p; B loader: k = 2 (t % 8)
    // + {0, 1} of columns t / 8 + 32 p
    constexpr int AP = (TM * BK) / 256;  // A elements per thread
    const int ar = t % TM, ak = t / TM;
    const int lk = 2 * (t & 7), lc = t >> 3;
    T ra[AP], rb[NT][2];
    auto load = [&](int kb) {
#pragma unroll
        for (int p = 0; p < AP; ++p) {
            const int k = kb + ak + (256 / TM) * p;
            const long r = r0 + ar;
            ra[p] = (k < M && r < K) ? A[r + (long)k * lda] : (T)0;
        }
#pragma unroll
        for (int p = 0; p < NT; ++p) {
            const int n = n0 + lc + 32 * p;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int k = kb + lk + u;
                rb[p][u] = (k < M && n < N) ? (T)Bm[k + (long)n * ldb] : (T)0;
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int p = 0; p < AP; ++p) sA[buf][(ak + (256 / TM) * p) * LA + ar] = ra[p];
#pragma unroll
        for (int p = 0; p < NT; ++p)
#pragma unroll
            for (int u = 0; u < 2; ++u) sB[buf][(lk + u) * LB + lc + 32 * p] = rb[p][u];
    };
    const int nst = (M + BK - 1) / BK;
    load(0);
    store(0);
    __syncthreads();
    for (int s = 0; s < nst; ++s) {
        const int buf = s & 1;
        if (s + 1 < nst) load((s + 1) * BK);
        mfma_stage<T, MT, NT>(sA[buf], LA, sB[buf], LB, wr0, wc0, lane, acc);
        if (s + 1 < nst) store(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long row = r0 + wr0 + 16 * i + Mfma<T>::row(lane, r);
                const int n = n0 + wc0 + 16 * j + (lane & 15);
                if (row < K && n < N) Out[row + (long)n * ldo] = acc[i][j][r];
            }
}

template <typename T, int NT, int MT = 2>
static sparc_status gemm_nn_launch(sparc_gpu_ctx c, long K, int N, int M, const T* A, long lda, const double* Bm,
                                   int ldb, T* Out, long ldo) {
    dim3 grid(div_up(K, 32 * MT), div_up(N, 32 * NT));
    const int slot = prof_begin(c, PK_GEMM_NN);
    k_gemm_nn<T, MT, NT><<<grid, 256, 0, c->stream>>>(K, N, M, A, lda, Bm, ldb, Out, ldo);
    SG_CHECK_LAUNCH(c);
    prof_end(c, slot);
    return SPARC_OK;
}

template <typename T>
sparc_status gemm_nn(sparc_gpu_ctx c, long K, int N, int M, const T* A, long lda, const double* Bm, int ldb, T* Out,
                     long ldo) {
    if (N <= 32) return gemm_nn_launch<T, 1>(c, K, N, M, A, lda, Bm, ldb, Out, ldo);
    if (N <= 96) return gemm_nn_launch<T, 3>(c, K, N, M, A, lda, Bm, ldb, Out, ldo);
    // 160-column tiles (two waves per SIMD) or 288-column (one per SIMD,
    // fewer passes over A); tuning override SPARC_GPU_GEMM_NN_COLS = 160 | 288.
    // Rows per tile: 128 for FP64 (twice the MFMAs per barrier: 92.6 against
    // 102.1 ms at 1.73M x 1200 x 1200), 64 for FP32 (71.1 against 73.5 ms);
    // override SPARC_GPU_GEMM_NN_ROWS = 64 | 128
    if (c->gemm_nn_cols == 288) return gemm_nn_launch<T, 9>(c, K, N, M, A, lda, Bm, ldb, Out, ldo);
    const int rows = c->gemm_nn_rows > 0 ? c->gemm_nn_rows : (sizeof(T) == 8 ? 128 : 64);
    if (rows == 128) return gemm_nn_launch<T, 5, 4>(c, K, N, M, A, lda, Bm, ldb, Out, ldo);
    return gemm_nn_launch<T, 5>(c, K, N, M, A, lda, Bm, ldb, Out, ldo);
}

template sparc_status gemm_tn<double>(sparc_gpu_ctx, int, int, long, const double*, long, const double*, long, double,
                                      double*, int, bool);
template sparc_status gemm_tn<float>(sparc_gpu_ctx, int, int, long, const float*, long, const float*, long, double,
                                     double*, int, bool);
template sparc_status gemm_nn<double>(sparc_gpu_ctx, long, int, int, const double*, long, const double*, int, double*,
                                      long);
template sparc_status gemm_nn<float>(sparc_gpu_ctx, long, int, int, const float*, long, const double*, int, float*,
                                     long);

}  // namespace sg
