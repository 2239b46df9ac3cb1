// Dense subspace products of Rayleigh-Ritz on MFMA (the Gram matrix
// dV Y^T Y, the projected Hamiltonian dV Y^T (H Y) and the rotation Y T).
//
// gemm_tn: C = alpha A^T B for tall-skinny A (K x M), B (K x N), K = N_d.
//   Deterministic split-K: each workgroup reduces one K-chunk of one 64x64
//   tile on MFMA (FP64 MFMA for double; FP32 MFMA with FP32 accumulation
//   inside the chunk for float) and writes a double partial; a second kernel
//   sums the partials in a fixed order in double.
// gemm_nn: Out = A Bm with A tall (K x M), Bm small (M x N, double, rounded
//   to the block precision), 64x64 output tiles.
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

constexpr int TB = 64;   // tile edge
constexpr int BK = 16;   // K per LDS stage
constexpr int PAD = 4;

// Partial[split][n][m] = sum_{k in chunk} A[k, m] B[k, n] for one tile.
template <typename T>
__global__ __launch_bounds__(256) void k_gemm_tn_split(int M, int N, long K, long kchunk, const T* __restrict__ A,
                                                       long lda, const T* __restrict__ B, long ldb,
                                                       double* __restrict__ part, int tiles_m, bool symmetric) {
    using acc_t = typename Mfma<T>::acc_t;
    __shared__ T sA[BK][TB + PAD];
    __shared__ T sB[BK][TB + PAD];
    const int tile = blockIdx.x;
    const int tm = tile % tiles_m, tn = tile / tiles_m;
    if (symmetric && tn < tm) return;
    const int split = blockIdx.y;
    const long k0 = (long)split * kchunk;
    const long k1 = min(K, k0 + kchunk);
    const int m0 = tm * TB, n0 = tn * TB;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wm = (wv & 1) * 32, wn = (wv >> 1) * 32;

    acc_t acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    // loader: thread t handles column (t / 4) of the tile, 4 consecutive k
    const int lcol = t >> 2, lk = (t & 3) * 4;
    const bool va = (m0 + lcol) < M, vb = (n0 + lcol) < N;
    const T* pa = A + (long)(m0 + (va ? lcol : 0)) * lda;
    const T* pb = B + (long)(n0 + (vb ? lcol : 0)) * ldb;

    for (long kb = k0; kb < k1; kb += BK) {
        T ra[4], rb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            long k = kb + lk + i;
            bool in = k < k1;
            ra[i] = (va && in) ? pa[k] : (T)0;
            rb[i] = (vb && in) ? pb[k] : (T)0;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            sA[lk + i][lcol] = ra[i];
            sB[lk + i][lcol] = rb[i];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            T av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) av[i] = sA[kk + (lane >> 4)][wm + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 2; ++j) bv[j] = sB[kk + (lane >> 4)][wn + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = Mfma<T>::run(av[i], bv[j], acc[i][j]);
        }
    }
    double* P = part + (long)split * M * N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int m = m0 + wm + i * 16 + Mfma<T>::row(lane, r);
                int n = n0 + wn + j * 16 + (lane & 15);
                if (m < M && n < N) P[m + (long)n * M] = (double)acc[i][j][r];
            }
}

__global__ void k_gemm_reduce(int M, int N, int nsplit, const double* __restrict__ part, double alpha,
                              double* __restrict__ C, int ldc, bool symmetric) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)M * N) return;
    int m = (int)(e % M), n = (int)(e / M);
    int sm = m, sn = n;
    if (symmetric && (n / TB) < (m / TB)) {
        sm = n;
        sn = m;
    }
    double s = 0.0;
    for (int k = 0; k < nsplit; ++k) s += part[(long)k * M * N + sm + (long)sn * M];
    C[m + (long)n * ldc] = alpha * s;
}

template <typename T>
sparc_status gemm_tn(sparc_gpu_ctx c, int M, int N, long K, const T* A, long lda, const T* B, long ldb,
                     double alpha, double* C, int ldc, bool symmetric) {
    if (symmetric && M != N) return set_err(c, SPARC_ERR_ARG, "gemm_tn: symmetric needs M == N");
    const int tiles_m = div_up(M, TB), tiles_n = div_up(N, TB);
    const int tiles = tiles_m * tiles_n;
    // enough workgroups to fill 256 CUs several times, chunks of >= 512 rows
    long want = std::max<long>(1, 2048 / tiles);
    long kchunk = std::max<long>(512, (K + want - 1) / want);
    kchunk = (kchunk + BK - 1) / BK * BK;
    int nsplit = (int)((K + kchunk - 1) / kchunk);
    sparc_status st = ensure_gemm_part(c, (size_t)nsplit * M * N);
    if (st != SPARC_OK) return st;
    dim3 grid(tiles, nsplit);
    const int slot = prof_begin(c, PK_GEMM_TN);
    k_gemm_tn_split<T><<<grid, 256, 0, c->stream>>>(M, N, K, kchunk, A, lda, B, ldb, c->gemm_part, tiles_m,
                                                  symmetric);
    SG_CHECK_LAUNCH(c);
    prof_end(c, slot);
    k_gemm_reduce<<<div_up((long)M * N, 256), 256, 0, c->stream>>>(M, N, nsplit, c->gemm_part, alpha, C, ldc,
                                                                   symmetric);
    SG_CHECK_LAUNCH(c);
    return SPARC_OK;
}

template <typename T>
__global__ __launch_bounds__(256) void k_gemm_nn(long K, int N, int M, const T* __restrict__ A, long lda,
                                                 const double* __restrict__ Bm, int ldb, T* __restrict__ Out,
                                                 long ldo) {
    using acc_t = typename Mfma<T>::acc_t;
    __shared__ T sA[BK][TB + PAD];
    __shared__ T sB[BK][TB + PAD];
    const long r0 = (long)blockIdx.x * TB;
    const int n0 = blockIdx.y * TB;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wm = (wv & 1) * 32, wn = (wv >> 1) * 32;
    acc_t acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
    // A loader: inner index t/16, 4 consecutive rows; B loader: inner t/16,
    // 4 consecutive output columns
    const int li = t >> 4, lr = (t & 15) * 4;
    for (int kb = 0; kb < M; kb += BK) {
        T ra[4], rb[4];
        const int ki = kb + li;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            long r = r0 + lr + i;
            ra[i] = (ki < M && r < K) ? A[r + (long)ki * lda] : (T)0;
            int n = n0 + lr + i;
            rb[i] = (ki < M && n < N) ? (T)Bm[ki + (long)n * ldb] : (T)0;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            sA[li][lr + i] = ra[i];
            sB[li][lr + i] = rb[i];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            T av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) av[i] = sA[kk + (lane >> 4)][wm + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 2; ++j) bv[j] = sB[kk + (lane >> 4)][wn + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = Mfma<T>::run(av[i], bv[j], acc[i][j]);
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                long row = r0 + wm + i * 16 + Mfma<T>::row(lane, r);
                int n = n0 + wn + j * 16 + (lane & 15);
                if (row < K && n < N) Out[row + (long)n * ldo] = acc[i][j][r];
            }
}

template <typename T>
sparc_status gemm_nn(sparc_gpu_ctx c, long K, int N, int M, const T* A, long lda, const double* Bm, int ldb, T* Out,
                     long ldo) {
    dim3 grid(div_up(K, TB), div_up(N, TB));
    const int slot = prof_begin(c, PK_GEMM_NN);
    k_gemm_nn<T><<<grid, 256, 0, c->stream>>>(K, N, M, A, lda, Bm, ldb, Out, ldo);
    SG_CHECK_LAUNCH(c);
    prof_end(c, slot);
    return SPARC_OK;
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
