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
    const int* pt_off;
    const int* pt_atom;
    const T* pt_chi;
    const T* D;       // gamma-scaled projections, column j at D + j*ldD
    int ldD;
    const double* params;  // a, b, a0 on the device
    int mode;              // 0: H x; 1: first filter step; 2: filter step `step`
    int step;
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

template <typename T, bool NL>
__global__ __launch_bounds__(1024) void k_hsweep(SweepArgs<T> a) {
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
    const int col = logical / a.ntiles_y;
    const int tile = logical - col * a.ntiles_y;
    const int y0 = tile * a.ty;
    const int tyn = min(a.ty, ny - y0);

    const int t = threadIdx.x;
    const int nt = blockDim.x;
    const int lx = t % nx, ly = t / nx;
    const bool active = ly < tyn;
    const long plane = (long)nx * ny;
    const T* __restrict__ xc = a.x + (long)col * a.ldx;
    T* oc = a.out + (long)col * a.ldx;
    const T* pc = a.xprev ? a.xprev + (long)col * a.ldx : nullptr;
    const long pxy = lx + (long)nx * (y0 + (active ? ly : 0));

    double alpha_d, c_d, beta_d;
    filter_coefs(a.params, a.mode, a.step, alpha_d, c_d, beta_d);
    const T alpha = (T)alpha_d, cshift = (T)c_d, beta = (T)beta_d;

    T q[2 * NO + 1];
#pragma unroll
    for (int j = 0; j <= 2 * NO; ++j) {
        int zz = j - NO;
        zz = zz < 0 ? zz + nz : zz;
        q[j] = active ? xc[pxy + (long)zz * plane] : (T)0;
    }

    const int nhalo = 2 * NO * nx;
    for (int z = 0; z < nz; ++z) {
        T* buf = (z & 1) ? buf1 : buf0;
        if (active) {
            T* row = buf + (ly + NO) * W + NO;
            row[lx] = q[NO];
            if (lx < NO) row[lx + nx] = q[NO];
            if (lx >= nx - NO) row[lx - nx] = q[NO];
        }
        const T* zp = xc + (long)z * plane;
        for (int e = t; e < nhalo; e += nt) {
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
            T v = zp[hx + (long)nx * gy];
            T* row = buf + lrow * W + NO;
            row[hx] = v;
            if (hx < NO) row[hx + nx] = v;
            if (hx >= nx - NO) row[hx - nx] = v;
        }
        __syncthreads();
        if (active) {
            const T* rp = buf + (ly + NO) * W + NO + lx;
            T lap = a.cf.c0 * q[NO];
#pragma unroll
            for (int k = 1; k <= NO; ++k) {
                lap += a.cf.cx[k] * (rp[k] + rp[-k]);
                lap += a.cf.cy[k] * (rp[k * W] + rp[-k * W]);
                lap += a.cf.cz[k] * (q[NO + k] + q[NO - k]);
            }
            const long p = pxy + (long)z * plane;
            T hv = lap + a.veff[p] * q[NO];
            if (NL) {
                const int e0 = a.pt_off[p], e1 = a.pt_off[p + 1];
                const T* Dc = a.D + (long)col * a.ldD;
                for (int e = e0; e < e1; ++e) {
                    const int at = 4 * a.pt_atom[e];
                    const T* ch = a.pt_chi + 4 * (long)e;
                    hv += ch[0] * Dc[at] + ch[1] * Dc[at + 1] + ch[2] * Dc[at + 2] + ch[3] * Dc[at + 3];
                }
            }
            T o;
            if (a.mode == 0) {
                o = hv;
            } else {
                o = alpha * (hv - cshift * q[NO]);
                if (a.mode == 2) o += beta * pc[p];
            }
            oc[p] = o;
        }
#pragma unroll
        for (int j = 0; j < 2 * NO; ++j) q[j] = q[j + 1];
        if (active) {
            int zn = z + NO + 1;
            zn = zn >= nz ? zn - nz : zn;
            q[2 * NO] = xc[pxy + (long)zn * plane];
        }
    }
}

// D(4a+lm, j) = gamma_lm * dV * sum_{s in support(a)} chi_lm(s) X(idx(s), j),
// accumulated in double in a fixed order (deterministic).
template <typename T, int NB>
__global__ __launch_bounds__(256) void k_projection(const T* __restrict__ x, long ldx, int ncol,
                                                    const long* __restrict__ sup_off, const int* __restrict__ sup_idx,
                                                    const double* __restrict__ chi, const double* __restrict__ g4,
                                                    double dV, T* __restrict__ D, int ldD) {
    const int a = blockIdx.x;
    const int n0 = blockIdx.y * NB;
    const int nb = min(NB, ncol - n0);
    double acc[NB][4];
#pragma unroll
    for (int n = 0; n < NB; ++n)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[n][k] = 0.0;
    const long s0 = sup_off[a], s1 = sup_off[a + 1];
    for (long s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
        const long idx = sup_idx[s];
        const double c0 = chi[4 * s], c1 = chi[4 * s + 1], c2 = chi[4 * s + 2], c3 = chi[4 * s + 3];
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            if (n < nb) {
                double v = (double)x[idx + (long)(n0 + n) * ldx];
                acc[n][0] += c0 * v;
                acc[n][1] += c1 * v;
                acc[n][2] += c2 * v;
                acc[n][3] += c3 * v;
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

static int choose_ty(int nx, int ny) {
    int maxty = std::max(1, std::min(16, 1024 / nx));
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
static const T* ptchi_of(sparc_gpu_ctx c);
template <>
const double* ptchi_of<double>(sparc_gpu_ctx c) {
    return c->nl.pt_chi;
}
template <>
const float* ptchi_of<float>(sparc_gpu_ctx c) {
    return c->nl.pt_chi32;
}

template <typename T>
sparc_status launch_hsweep(sparc_gpu_ctx c, const T* x, T* out, const T* xprev, int ncol, long ldx, int mode,
                           int step) {
    SweepArgs<T> a;
    a.x = x;
    a.out = out;
    a.xprev = xprev;
    a.ldx = ldx;
    a.nx = c->nx;
    a.ny = c->ny;
    a.nz = c->nz;
    a.ty = choose_ty(c->nx, c->ny);
    a.ntiles_y = div_up(c->ny, a.ty);
    a.cf = coef<T>(c);
    a.veff = veff_of<T>(c);
    const bool nl = c->nl_lmax >= 1 && c->nl.n_sup > 0;
    a.pt_off = c->nl.pt_off;
    a.pt_atom = c->nl.pt_atom;
    a.pt_chi = ptchi_of<T>(c);
    a.D = D_of<T>(c);
    a.ldD = 4 * c->n_atoms;
    a.params = c->scal + S_A;
    a.mode = mode;
    a.step = step;
    const int threads = div_up((long)c->nx * a.ty, 64) * 64;
    const size_t shmem = 2 * (size_t)(a.ty + 2 * kMaxHalfOrder) * (c->nx + 2 * kMaxHalfOrder) * sizeof(T);
    const long nblocks = (long)ncol * a.ntiles_y;
    if (nblocks > 0x7fffffffL) return set_err(c, SPARC_ERR_ARG, "too many blocks");
    if (nl)
        k_hsweep<T, true><<<(int)nblocks, threads, shmem, c->stream>>>(a);
    else
        k_hsweep<T, false><<<(int)nblocks, threads, shmem, c->stream>>>(a);
    SG_CHECK_LAUNCH(c);
    return SPARC_OK;
}

template <typename T>
sparc_status launch_projection(sparc_gpu_ctx c, const T* x, int ncol, long ldx) {
    if (c->nl_lmax < 1 || c->nl.n_sup == 0) return SPARC_OK;
    constexpr int NB = 8;
    dim3 grid(c->n_atoms, div_up(ncol, NB));
    k_projection<T, NB><<<grid, 256, 0, c->stream>>>(x, ldx, ncol, c->nl.sup_off, c->nl.sup_idx, c->nl.sup_chi,
                                                   c->nl.gamma4, c->dV, D_of<T>(c), 4 * c->n_atoms);
    SG_CHECK_LAUNCH(c);
    return SPARC_OK;
}

template sparc_status launch_hsweep<double>(sparc_gpu_ctx, const double*, double*, const double*, int, long, int,
                                            int);
template sparc_status launch_hsweep<float>(sparc_gpu_ctx, const float*, float*, const float*, int, long, int, int);
template sparc_status launch_projection<double>(sparc_gpu_ctx, const double*, int, long);
template sparc_status launch_projection<float>(sparc_gpu_ctx, const float*, int, long);

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
template <typename T>
sparc_status filter_impl(sparc_gpu_ctx c, T* X, T* Wk, int ncol, long ldx, int m) {
    sparc_status st;
    if ((st = launch_projection<T>(c, X, ncol, ldx)) != SPARC_OK) return st;
    if ((st = launch_hsweep<T>(c, X, Wk, nullptr, ncol, ldx, 1, 1)) != SPARC_OK) return st;
    for (int k = 2; k <= m; ++k) {
        T* cur = (k % 2 == 0) ? Wk : X;   // Y_{k-1}
        T* dst = (k % 2 == 0) ? X : Wk;   // Y_{k-2}, overwritten with Y_k
        if ((st = launch_projection<T>(c, cur, ncol, ldx)) != SPARC_OK) return st;
        if ((st = launch_hsweep<T>(c, cur, dst, dst, ncol, ldx, 2, k)) != SPARC_OK) return st;
    }
    if (m % 2 == 1) {
        dim3 grid(div_up(c->nd, 256), ncol);
        k_copy_block<T><<<grid, 256, 0, c->stream>>>(Wk, X, c->nd, ncol, ldx);
        SG_CHECK_LAUNCH(c);
    }
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
__global__ void k_bounds(const double* v, long n, double kin, double nl_lo, double nl_hi, double* out_lo,
                         double* out_hi) {
    __shared__ double smin[1024], smax[1024];
    double mn = 1e300, mx = -1e300;
    for (long i = threadIdx.x; i < n; i += blockDim.x) {
        double x = v[i];
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
        *out_lo = smin[0] + nl_lo;
        *out_hi = kin + smax[0] + nl_hi;
    }
}

sparc_status bounds_impl(sparc_gpu_ctx c) {
    k_bounds<<<1, 1024, 0, c->stream>>>(c->veff, c->nd, c->kin_bound, c->nl.nl_lo, c->nl.nl_hi, c->scal + S_LO,
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
