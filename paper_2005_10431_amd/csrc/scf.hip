// SCF iteration around CheFSI (Sec. 2.1): potential from the density,
// filter + Rayleigh-Ritz passes, Fermi-Dirac occupations, density
// (Sec. 2 eq. (2)), free energy, residual and linear mixing.
//
// Electrostatics: -Delta_h phi = 4 pi (rho + b - mean) on the periodic grid.
// The discrete periodic Laplacian is separable and each 1D stencil is
// diagonalised by a real orthonormal Fourier basis U_d, so
//   phi = (U_z x U_y x U_x) diag(4 pi / lambda) (U_z x U_y x U_x)^T (rho + b)
// with lambda the eigenvalues of -Delta_h and the constant mode dropped.  This
// is the exact solution of the same linear system the paper's iterative
// stencil solver (AAR) converges to; here it costs six small dense
// transforms along the grid axes.
#include <cmath>
#include <cstring>

#include "internal.hpp"

namespace sg {

// out = (I x M x I) in along `axis`, M = U^T (fwd) or U (bwd); U is n x n
// column-major (column k = mode k).
__global__ void k_axis_transform(const double* __restrict__ in, double* __restrict__ out,
                                 const double* __restrict__ U, int nx, int ny, int nz, int axis, int fwd) {
    long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long nd = (long)nx * ny * nz;
    if (p >= nd) return;
    int ix = (int)(p % nx);
    int iy = (int)((p / nx) % ny);
    int iz = (int)(p / ((long)nx * ny));
    int n, m;
    long stride, base;
    if (axis == 0) {
        n = nx;
        m = ix;
        stride = 1;
        base = p - ix;
    } else if (axis == 1) {
        n = ny;
        m = iy;
        stride = nx;
        base = p - (long)iy * nx;
    } else {
        n = nz;
        m = iz;
        stride = (long)nx * ny;
        base = p - (long)iz * nx * ny;
    }
    double acc = 0.0;
    if (fwd) {
        const double* u = U + (long)m * n;  // column m of U = row m of U^T
        for (int l = 0; l < n; ++l) acc += u[l] * in[base + l * stride];
    } else {
        for (int l = 0; l < n; ++l) acc += U[m + (long)l * n] * in[base + l * stride];
    }
    out[p] = acc;
}

__global__ void k_add(const double* a, const double* b, double* out, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] + b[i];
}

__global__ void k_mul(double* a, const double* b, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] *= b[i];
}

// Unpolarised LDA: Slater exchange and the PW92 correlation fit.
__device__ inline void lda_point(double rho, double floor_, double& exc, double& vxc) {
    const double pi = 3.14159265358979323846;
    double r = fmax(rho, floor_);
    double ex = -0.75 * cbrt(3.0 * r / pi);
    double vx = (4.0 / 3.0) * ex;
    double rs = cbrt(3.0 / (4.0 * pi * r));
    const double A = 0.031091, a1 = 0.21370, b1 = 7.5957, b2 = 3.5876, b3 = 1.6382, b4 = 0.49294;
    double srs = sqrt(rs);
    double Q0 = -2.0 * A * (1.0 + a1 * rs);
    double Q1 = 2.0 * A * (b1 * srs + b2 * rs + b3 * rs * srs + b4 * rs * rs);
    double dQ1 = A * (b1 / srs + 2.0 * b2 + 3.0 * b3 * srs + 4.0 * b4 * rs);
    double lg = log1p(1.0 / Q1);
    double ec = Q0 * lg;
    double dec = -2.0 * A * a1 * lg - Q0 * dQ1 / (Q1 * Q1 + Q1);
    exc = ex + ec;
    vxc = vx + ec - rs / 3.0 * dec;
}

__global__ void k_lda(const double* __restrict__ rho, const double* __restrict__ phi, double floor_,
                      double* __restrict__ exc, double* __restrict__ vxc, double* __restrict__ veff,
                      float* __restrict__ veff32, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double e, v;
    lda_point(rho[i], floor_, e, v);
    if (exc) exc[i] = e;
    if (vxc) vxc[i] = v;
    if (veff) {
        double ve = phi[i] + v;
        veff[i] = ve;
        if (veff32) veff32[i] = (float)ve;
    }
}

// phi, eps_xc, v_xc, V_eff for density rho.  Uses fields[0..1] as scratch;
// phi may not be null inside (a field is substituted).
sparc_status potential_impl(sparc_gpu_ctx c, const double* rho, double* phi, double* exc, double* vxc,
                            double* veff) {
    sparc_status st = ensure_fields(c, 6);
    if (st != SPARC_OK) return st;
    double* t0 = c->field;
    double* t1 = c->field + c->nd;
    double* ph = phi ? phi : c->field + 2 * c->nd;
    const int nb = div_up(c->nd, 256);
    k_add<<<nb, 256, 0, c->stream>>>(rho, c->b, t0, c->nd);
    k_axis_transform<<<nb, 256, 0, c->stream>>>(t0, t1, c->pois_ux, c->nx, c->ny, c->nz, 0, 1);
    k_axis_transform<<<nb, 256, 0, c->stream>>>(t1, t0, c->pois_uy, c->nx, c->ny, c->nz, 1, 1);
    k_axis_transform<<<nb, 256, 0, c->stream>>>(t0, t1, c->pois_uz, c->nx, c->ny, c->nz, 2, 1);
    k_mul<<<nb, 256, 0, c->stream>>>(t1, c->pois_inv, c->nd);
    k_axis_transform<<<nb, 256, 0, c->stream>>>(t1, t0, c->pois_uz, c->nx, c->ny, c->nz, 2, 0);
    k_axis_transform<<<nb, 256, 0, c->stream>>>(t0, t1, c->pois_uy, c->nx, c->ny, c->nz, 1, 0);
    k_axis_transform<<<nb, 256, 0, c->stream>>>(t1, ph, c->pois_ux, c->nx, c->ny, c->nz, 0, 0);
    float* v32 = (veff == c->veff) ? c->veff32 : nullptr;
    k_lda<<<nb, 256, 0, c->stream>>>(rho, ph, c->rho_floor, exc, vxc, veff, v32, c->nd);
    SG_CHECK_LAUNCH(c);
    return SPARC_OK;
}

// ---- spin-polarised LDA --------------------------------------------------
// Exchange: E_x[rho_up, rho_dn] = (E_x[2 rho_up] + E_x[2 rho_dn]) / 2.
// Correlation: PW92 interpolation in zeta between the unpolarised fit, the
// fully polarised fit and the spin stiffness alpha_c (all of the form G).

__device__ inline void pw92_form(double rs, double srs, double A, double a1, double b1, double b2, double b3,
                                 double b4, double& G, double& dG) {
    const double Q0 = -2.0 * A * (1.0 + a1 * rs);
    const double Q1 = 2.0 * A * (b1 * srs + b2 * rs + b3 * rs * srs + b4 * rs * rs);
    const double dQ1 = A * (b1 / srs + 2.0 * b2 + 3.0 * b3 * srs + 4.0 * b4 * rs);
    const double lg = log1p(1.0 / Q1);
    G = Q0 * lg;
    dG = -2.0 * A * a1 * lg - Q0 * dQ1 / (Q1 * Q1 + Q1);
}

__device__ inline void lsda_point(double ru, double rd, double floor_, double& exc, double& vu, double& vd) {
    const double pi = 3.14159265358979323846;
    ru = fmax(ru, 0.5 * floor_);
    rd = fmax(rd, 0.5 * floor_);
    const double r = ru + rd;
    const double z = (ru - rd) / r;
    const double exu = -0.75 * cbrt(6.0 * ru / pi);
    const double exd = -0.75 * cbrt(6.0 * rd / pi);
    const double ex = (ru * exu + rd * exd) / r;
    const double rs = cbrt(3.0 / (4.0 * pi * r));
    const double srs = sqrt(rs);
    double e0, d0, e1, d1, ma, dma;
    pw92_form(rs, srs, 0.031091, 0.21370, 7.5957, 3.5876, 1.6382, 0.49294, e0, d0);
    pw92_form(rs, srs, 0.015545, 0.20548, 14.1189, 6.1977, 3.3662, 0.62517, e1, d1);
    pw92_form(rs, srs, 0.016887, 0.11125, 10.357, 3.6231, 0.88026, 0.49671, ma, dma);
    const double ac = -ma, dac = -dma;
    const double fden = 0.51984209978974632953;     // 2^(4/3) - 2
    const double fz20 = 8.0 / (9.0 * fden);          // f''(0)
    const double up = 1.0 + z, dn = 1.0 - z;
    const double cu = cbrt(up), cd = cbrt(dn);
    const double f = (up * cu + dn * cd - 2.0) / fden;
    const double df = (4.0 / 3.0) * (cu - cd) / fden;
    const double z3 = z * z * z, z4 = z3 * z;
    const double ec = e0 + ac * f / fz20 * (1.0 - z4) + (e1 - e0) * f * z4;
    const double dec_rs = d0 + dac * f / fz20 * (1.0 - z4) + (d1 - d0) * f * z4;
    const double dec_z = ac / fz20 * (df * (1.0 - z4) - 4.0 * z3 * f) + (e1 - e0) * (df * z4 + 4.0 * z3 * f);
    const double common = ec - rs / 3.0 * dec_rs;
    exc = ex + ec;
    vu = (4.0 / 3.0) * exu + common + (1.0 - z) * dec_z;
    vd = (4.0 / 3.0) * exd + common - (1.0 + z) * dec_z;
}

// rho: 2 n (up, down); vxc, veff: 2 n (may be null); exc: n (may be null)
__global__ void k_lsda(const double* __restrict__ rho, const double* __restrict__ phi, double floor_,
                       double* __restrict__ exc, double* __restrict__ vxc, double* __restrict__ veff, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double e, vu, vd;
    lsda_point(rho[i], rho[n + i], floor_, e, vu, vd);
    if (exc) exc[i] = e;
    if (vxc) {
        vxc[i] = vu;
        vxc[n + i] = vd;
    }
    if (veff) {
        veff[i] = phi[i] + vu;
        veff[n + i] = phi[i] + vd;
    }
}

__global__ void k_add3(const double* a, const double* b, const double* c, double* out, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (a[i] + b[i]) + c[i];
}

// phi of the total density, eps_xc, v_xc and V_eff of both spins.  Uses
// fields[0..1] as scratch (phi falls back to field 2).
static sparc_status potential_spin_impl(sparc_gpu_ctx c, const double* rho, double* phi, double* exc, double* vxc,
                                        double* veff) {
    sparc_status st = ensure_fields(c, 3);
    if (st != SPARC_OK) return st;
    const long nd = c->nd;
    double* t0 = c->field;
    double* t1 = c->field + nd;
    double* ph = phi ? phi : c->field + 2 * nd;
    const int nb = div_up(nd, 256);
    k_add3<<<nb, 256, 0, c->stream>>>(rho, rho + nd, c->b, t0, nd);
    k_axis_transform<<<nb, 256, 0, c->stream>>>(t0, t1, c->pois_ux, c->nx, c->ny, c->nz, 0, 1);
    k_axis_transform<<<nb, 256, 0, c->stream>>>(t1, t0, c->pois_uy, c->nx, c->ny, c->nz, 1, 1);
    k_axis_transform<<<nb, 256, 0, c->stream>>>(t0, t1, c->pois_uz, c->nx, c->ny, c->nz, 2, 1);
    k_mul<<<nb, 256, 0, c->stream>>>(t1, c->pois_inv, nd);
    k_axis_transform<<<nb, 256, 0, c->stream>>>(t1, t0, c->pois_uz, c->nx, c->ny, c->nz, 2, 0);
    k_axis_transform<<<nb, 256, 0, c->stream>>>(t0, t1, c->pois_uy, c->nx, c->ny, c->nz, 1, 0);
    k_axis_transform<<<nb, 256, 0, c->stream>>>(t1, ph, c->pois_ux, c->nx, c->ny, c->nz, 0, 0);
    k_lsda<<<nb, 256, 0, c->stream>>>(rho, ph, c->rho_floor, exc, vxc, veff, nd);
    SG_CHECK_LAUNCH(c);
    return SPARC_OK;
}

// ------------------------------------------------------------ occupations

__device__ inline double fermi(double lam, double mu, double kT) {
    double x = (lam - mu) / kT;
    if (x > 0.0) {
        double e = exp(-x);
        return e / (1.0 + e);
    }
    return 1.0 / (1.0 + exp(x));
}

// One block: bisection for mu, then occupations g = deg f and the entropy
// term: out[0] = mu, out[1] = deg kT sum [f ln f + (1-f) ln(1-f)],
// out[2] = sum g lam.  deg = 2 spin-unpolarised, 1 per spin state.
__global__ __launch_bounds__(256) void k_occupations(const double* __restrict__ eig, int N, double ne, double kT,
                                                     double deg, const double* __restrict__ wts,
                                                     double* __restrict__ occ, double* __restrict__ out,
                                                     int* __restrict__ flag) {
    __shared__ double red[256];
    __shared__ double s_lo, s_hi, s_mu;
    __shared__ int s_done;
    const int t = threadIdx.x;
    if (t == 0) {
        s_lo = eig[0] - 40.0 * kT;
        s_hi = eig[N - 1] + 40.0 * kT;
        s_done = 0;
        for (int i = 0; i < N; ++i) {
            s_lo = fmin(s_lo, eig[i] - 40.0 * kT);
            s_hi = fmax(s_hi, eig[i] + 40.0 * kT);
        }
    }
    __syncthreads();
    for (int it = 0; it < 500; ++it) {
        double mu = 0.5 * (s_lo + s_hi);
        double acc = 0.0;
        for (int i = t; i < N; i += blockDim.x) acc += deg * (wts ? wts[i] : 1.0) * fermi(eig[i], mu, kT);
        red[t] = acc;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (t < s) red[t] += red[t + s];
            __syncthreads();
        }
        if (t == 0) {
            double n = red[0];
            s_mu = mu;
            if (fabs(n - ne) < 1e-13) {
                s_done = 1;
            } else {
                if (n < ne)
                    s_lo = mu;
                else
                    s_hi = mu;
                double mid = 0.5 * (s_lo + s_hi);
                if (!(s_lo < mid && mid < s_hi)) s_done = 1;
            }
        }
        __syncthreads();
        if (s_done) break;
    }
    const double mu = s_mu;
    double ent = 0.0, band = 0.0;
    for (int i = t; i < N; i += blockDim.x) {
        double f = fermi(eig[i], mu, kT);
        const double wi = wts ? wts[i] : 1.0;
        occ[i] = deg * f;
        band += wi * deg * f * eig[i];
        if (f > 0.0 && f < 1.0) ent += wi * (f * log(f) + (1.0 - f) * log(1.0 - f));
    }
    __syncthreads();
    red[t] = ent;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    double ent_sum = red[0];
    __syncthreads();
    red[t] = band;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    if (t == 0) {
        out[0] = mu;
        out[1] = deg * kT * ent_sum;
        out[2] = red[0];
        if (!s_done || !isfinite(mu)) flag[0] = 1;
    }
}

sparc_status occupations_impl(sparc_gpu_ctx c, const double* eig, int ncol, double* occ, double* mu, double deg,
                              const double* wts) {
    k_occupations<<<1, 256, 0, c->stream>>>(eig, ncol, c->n_electrons, c->kT, deg, wts, occ, c->scal + S_OCC,
                                           c->flags + F_FERMI);
    SG_CHECK_LAUNCH(c);
    if (mu) SG_HIP(c, hipMemcpyAsync(mu, c->scal + S_OCC, sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return SPARC_OK;
}

// ------------------------------------------------------------ density

template <typename T>
__global__ __launch_bounds__(256) void k_density(const T* __restrict__ X, int ncol, long ldx,
                                                 const double* __restrict__ occ, double* __restrict__ rho, long nd) {
    long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nd) return;
    double acc = 0.0;
    for (int j = 0; j < ncol; ++j) {
        double v = (double)X[p + (long)j * ldx];
        acc += occ[j] * v * v;
    }
    rho[p] = acc;
}

template <typename T>
sparc_status density_impl(sparc_gpu_ctx c, const T* X, int ncol, long ldx, const double* occ, double* rho) {
    const int slot = prof_begin(c, PK_DENSITY);
    k_density<T><<<div_up(c->nd, 256), 256, 0, c->stream>>>(X, ncol, ldx, occ, rho, c->nd);
    SG_CHECK_LAUNCH(c);
    prof_end(c, slot);
    return SPARC_OK;
}
template sparc_status density_impl<double>(sparc_gpu_ctx, const double*, int, long, const double*, double*);
template sparc_status density_impl<float>(sparc_gpu_ctx, const float*, int, long, const double*, double*);

// ------------------------------------------------------------ energy + mixing

constexpr int kRed = 6;  // rho exc, rho vxc, (b - rho) phi, |dr|^2, |rho_out|^2, sum rho_out

// Per-block partial sums; optionally rho_in <- rho_in + beta (rho_out - rho_in).
__global__ __launch_bounds__(256) void k_energy_mix(double* __restrict__ rho_in, const double* __restrict__ rho_out,
                                                    const double* __restrict__ exc, const double* __restrict__ vxc,
                                                    const double* __restrict__ phi, const double* __restrict__ b,
                                                    long n, double beta, int do_mix, double* __restrict__ part) {
    __shared__ double red[kRed][256];
    const int t = threadIdx.x;
    double s[kRed] = {0, 0, 0, 0, 0, 0};
    for (long i = (long)blockIdx.x * blockDim.x + t; i < n; i += (long)gridDim.x * blockDim.x) {
        double ri = rho_in[i], ro = rho_out[i];
        s[0] += ri * exc[i];
        s[1] += ri * vxc[i];
        s[2] += (b[i] - ri) * phi[i];
        double d = ro - ri;
        s[3] += d * d;
        s[4] += ro * ro;
        s[5] += ro;
        if (do_mix) rho_in[i] = ri + beta * d;
    }
    for (int k = 0; k < kRed; ++k) red[k][t] = s[k];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (t < st)
            for (int k = 0; k < kRed; ++k) red[k][t] += red[k][t + st];
        __syncthreads();
    }
    if (t < kRed) part[(long)blockIdx.x * kRed + t] = red[t][0];
}

// The same partial sums for spin densities (2 nd vectors, up then down):
// rho exc with the total rho, sum_s rho_s vxc_s, (b - rho) phi, and the
// residual sums over both spins.
__global__ __launch_bounds__(256) void k_energy_spin(const double* __restrict__ rin, const double* __restrict__ rout,
                                                     const double* __restrict__ exc, const double* __restrict__ vxc,
                                                     const double* __restrict__ phi, const double* __restrict__ b,
                                                     long nd, double* __restrict__ part) {
    __shared__ double red[kRed][256];
    const int t = threadIdx.x;
    double s[kRed] = {0, 0, 0, 0, 0, 0};
    for (long i = (long)blockIdx.x * blockDim.x + t; i < nd; i += (long)gridDim.x * blockDim.x) {
        const double ru = rin[i], rd = rin[nd + i], ou = rout[i], od = rout[nd + i];
        const double r = ru + rd;
        s[0] += r * exc[i];
        s[1] += ru * vxc[i] + rd * vxc[nd + i];
        s[2] += (b[i] - r) * phi[i];
        const double du = ou - ru, dd = od - rd;
        s[3] += du * du + dd * dd;
        s[4] += ou * ou + od * od;
        s[5] += ou + od;
    }
    for (int k = 0; k < kRed; ++k) red[k][t] = s[k];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (t < st)
            for (int k = 0; k < kRed; ++k) red[k][t] += red[k][t + st];
        __syncthreads();
    }
    if (t < kRed) part[(long)blockIdx.x * kRed + t] = red[t][0];
}

__global__ void k_residual(const double* a, const double* b, double* out, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] - b[i];
}

// Eigencomponent scaling of the mixing preconditioner: the Poisson table
// holds 4 pi / lambda (0 for the constant mode), so
// lambda / (lambda + q0^2) = 4 pi / (4 pi + q0^2 inv); the constant mode is
// removed.
__global__ void k_kerker(double* t, const double* inv, double q02, long n) {
    const double fourpi = 12.566370614359172;
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) t[i] = (inv[i] == 0.0) ? 0.0 : t[i] * (fourpi / (fourpi + q02 * inv[i]));
}

__global__ void k_axpy(double* y, const double* x, double a, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += a * x[i];
}

// ---- periodic Pulay mixing (Sec. 2.1) --------------------------------------
// History buffer of N_d-vectors: [x_prev | f_prev | dX slots | dF slots].

static_assert(S_PULAY + SPARC_PULAY_MAX <= S_SPINB && S_SPINB + 6 <= S_COUNT, "scalar block layout");

// Which slots hold valid pairs at iteration `iter`, where this iteration's
// pair goes, and whether it is a Pulay iteration: the schedule is replayed
// from iteration 0 (the history buffer carries no bookkeeping of its own).
struct PulayPlan {
    int push_slot;   // -1 on iteration 0
    int count;       // valid pairs after this iteration's push
    int slots[SPARC_PULAY_MAX];
    bool pulay;
};

static PulayPlan pulay_plan(int iter, int m, int period, int restart) {
    PulayPlan p{};
    long pushes = 0;
    int cnt = 0;
    for (int k = 0; k <= iter; ++k) {
        int slot = -1;
        if (k >= 1) {
            slot = (int)(pushes % m);
            ++pushes;
            cnt = std::min(cnt + 1, m);
        }
        const bool pul = cnt > 0 && (k + 1) % period == 0;
        if (k == iter) {
            p.push_slot = slot;
            p.count = cnt;
            for (int j = 0; j < cnt; ++j) p.slots[j] = (int)((pushes - 1 - j) % m);
            p.pulay = pul;
        }
        if (pul && restart && cnt == m) cnt = 0;
    }
    return p;
}

struct SlotList {
    int s[SPARC_PULAY_MAX];
};

// x = rho_in, f = rho_out - rho_in; slot >= 0 receives dX = x - x_prev and
// dF = f - f_prev; then x_prev, f_prev <- x, f.
__global__ void k_pulay_push(const double* __restrict__ x, const double* __restrict__ ro, double* __restrict__ hist,
                             long nd, int m, int slot) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nd) return;
    const double xi = x[i], fi = ro[i] - xi;
    if (slot >= 0) {
        hist[(2 + slot) * nd + i] = xi - hist[i];
        hist[(2 + (long)m + slot) * nd + i] = fi - hist[nd + i];
    }
    hist[i] = xi;
    hist[nd + i] = fi;
}

// Per-block partial sums of the normal equations: the upper triangle of
// dF^T dF (row-major, a <= b) followed by dF^T f, for the C listed slots.
// Fixed-order reduction (wave shuffles, then the 4 waves in order).
template <int C>
__global__ __launch_bounds__(256) void k_pulay_dots(const double* __restrict__ hist, long nd, int m, SlotList sl,
                                                    double* __restrict__ part) {
    constexpr int P = C * (C + 1) / 2 + C;
    const double* f = hist + nd;
    const double* dF[C];
#pragma unroll
    for (int a = 0; a < C; ++a) dF[a] = hist + (2 + (long)m + sl.s[a]) * nd;
    double acc[P];
#pragma unroll
    for (int q = 0; q < P; ++q) acc[q] = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nd; i += (long)gridDim.x * blockDim.x) {
        double v[C];
#pragma unroll
        for (int a = 0; a < C; ++a) v[a] = dF[a][i];
        const double fi = f[i];
        int q = 0;
#pragma unroll
        for (int a = 0; a < C; ++a)
#pragma unroll
            for (int b = a; b < C; ++b) acc[q++] += v[a] * v[b];
#pragma unroll
        for (int a = 0; a < C; ++a) acc[q++] += v[a] * fi;
    }
    __shared__ double wsum[4][P];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        double t = acc[q];
        for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
        if (lane == 0) wsum[w][q] = t;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < P; q += blockDim.x)
        part[(long)blockIdx.x * P + q] = ((wsum[0][q] + wsum[1][q]) + wsum[2][q]) + wsum[3][q];
}

// Sum the block partials in block order, then solve the C x C normal
// equations by Gaussian elimination with partial pivoting (one thread).
// gamma -> scal[S_PULAY..]; a zero pivot or a non-finite gamma raises the
// flag and leaves gamma = 0.
__global__ __launch_bounds__(256) void k_pulay_solve(const double* __restrict__ part, int nblk, int C,
                                                     double* __restrict__ scal, int* __restrict__ flags) {
    constexpr int PM = SPARC_PULAY_MAX * (SPARC_PULAY_MAX + 1) / 2 + SPARC_PULAY_MAX;
    __shared__ double red[PM];
    __shared__ double A[SPARC_PULAY_MAX][SPARC_PULAY_MAX + 1];
    const int P = C * (C + 1) / 2 + C;
    const int t = threadIdx.x;
    if (t < P) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += part[(long)b * P + t];
        red[t] = s;
    }
    __syncthreads();
    if (t != 0) return;
    int q = 0;
    for (int a = 0; a < C; ++a)
        for (int b = a; b < C; ++b) {
            A[a][b] = red[q];
            A[b][a] = red[q];
            ++q;
        }
    for (int a = 0; a < C; ++a) A[a][C] = red[q++];
    bool bad = false;
    for (int k = 0; k < C && !bad; ++k) {
        int piv = k;
        for (int r = k + 1; r < C; ++r)
            if (fabs(A[r][k]) > fabs(A[piv][k])) piv = r;
        if (!(fabs(A[piv][k]) > 0.0)) {
            bad = true;
            break;
        }
        if (piv != k)
            for (int j = k; j <= C; ++j) {
                const double tmp = A[k][j];
                A[k][j] = A[piv][j];
                A[piv][j] = tmp;
            }
        for (int r = k + 1; r < C; ++r) {
            const double l = A[r][k] / A[k][k];
            for (int j = k; j <= C; ++j) A[r][j] -= l * A[k][j];
        }
    }
    double g[SPARC_PULAY_MAX];
    for (int k = C - 1; k >= 0 && !bad; --k) {
        double s = A[k][C];
        for (int j = k + 1; j < C; ++j) s -= A[k][j] * g[j];
        g[k] = s / A[k][k];
        if (!isfinite(g[k])) bad = true;
    }
    for (int k = 0; k < C; ++k) scal[S_PULAY + k] = bad ? 0.0 : g[k];
    if (bad) flags[F_PULAY_SINGULAR] = 1;
}

// x_bar = x - dX gamma, f_bar = f - dF gamma (sums formed first, in slot
// order); then x <- x_bar + beta f_bar, or x <- x_bar and t <- f_bar when the
// residual is still to be preconditioned (t != nullptr).
__global__ void k_pulay_apply(double* __restrict__ x, const double* __restrict__ hist, const double* __restrict__ scal,
                              long nd, int m, SlotList sl, int C, double beta, double* __restrict__ t) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nd) return;
    double sx = 0.0, sf = 0.0;
    for (int a = 0; a < C; ++a) {
        const double g = scal[S_PULAY + a];
        sx += hist[(2 + (long)sl.s[a]) * nd + i] * g;
        sf += hist[(2 + (long)m + sl.s[a]) * nd + i] * g;
    }
    const double xb = hist[i] - sx;
    const double fb = hist[nd + i] - sf;
    if (t) {
        x[i] = xb;
        t[i] = fb;
    } else {
        x[i] = xb + beta * fb;
    }
}

// Spin mixing vector f = [f_up; f_dn] (f = a - b, or f = a when b is
// null): sum <- f_up + f_dn, diff <- f_up - f_dn.  diff may alias a.
__global__ void k_spin_split(const double* a, const double* b, double* __restrict__ sum, double* diff, long nd) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nd) return;
    const double fu = b ? a[i] - b[i] : a[i];
    const double fd = b ? a[nd + i] - b[nd + i] : a[nd + i];
    sum[i] = fu + fd;
    diff[i] = fu - fd;
}

// x_up += beta (P sum + diff) / 2, x_dn += beta (P sum - diff) / 2
__global__ void k_spin_combine(double* __restrict__ x, const double* __restrict__ psum,
                               const double* __restrict__ diff, double beta, long nd) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nd) return;
    x[i] += beta * (0.5 * (psum[i] + diff[i]));
    x[nd + i] += beta * (0.5 * (psum[i] - diff[i]));
}

__global__ void k_mix_linear(double* __restrict__ x, const double* __restrict__ ro, double beta, long nd) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nd) {
        const double xi = x[i];
        x[i] = xi + beta * (ro[i] - xi);
    }
}

// out[q] = sum over blocks of part[i][q]: block q, fixed-order tree.
__global__ __launch_bounds__(256) void k_energy_final(const double* __restrict__ part, int nblk,
                                                      double* __restrict__ out) {
    __shared__ double red[256];
    const int q = blockIdx.x, t = threadIdx.x;
    double s = 0.0;
    for (int i = t; i < nblk; i += blockDim.x) s += part[(long)i * kRed + q];
    red[t] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (t < st) red[t] += red[t + st];
        __syncthreads();
    }
    if (t == 0) out[q] = red[0];
}

// filter bounds from the latest Ritz values: a = max, a0 = min (or the lower
// spectrum bound before the first filter); b = upper spectrum bound
__global__ void k_bounds_from_eig(const double* eig, int N, double* scal, int first) {
    scal[S_A] = eig[N - 1];
    scal[S_A0] = first ? scal[S_LO] : eig[0];
    scal[S_B] = scal[S_HI];
}

__global__ void k_set_ab(double* scal, double a, double a0) {
    scal[S_A] = a;
    scal[S_A0] = a0;
    scal[S_B] = scal[S_HI];
}

__global__ void k_set_b(double* scal) { scal[S_B] = scal[S_HI]; }

template <typename T>
__global__ void k_promote(const T* __restrict__ src, double* __restrict__ dst, long nd, int ncol, long lds, long ldd) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    if (i < nd) dst[i + (long)j * ldd] = (double)src[i + (long)j * lds];
}

// Events of one SCF call: recorded on the context stream while its work is
// enqueued and read after the call's single synchronisation.  The pool
// (c->step_ev) is grown by ensure_step_events before the first mark.
struct StepEvents {
    sparc_gpu_ctx c;
    int used = 0;
    explicit StepEvents(sparc_gpu_ctx cc) : c(cc) {}
    int mark() {
        if (used >= (int)c->step_ev.size()) return -1;
        hipEventRecord(c->step_ev[used], c->stream);
        return used++;
    }
    double ms(int a, int b) const {
        if (a < 0 || b < 0) return 0.0;
        float v = 0.f;
        hipEventElapsedTime(&v, c->step_ev[a], c->step_ev[b]);
        return (double)v;
    }
};

static sparc_status ensure_step_events(sparc_gpu_ctx c, int n) {
    while ((int)c->step_ev.size() < n) {
        hipEvent_t e = nullptr;
        SG_HIP(c, hipEventCreate(&e));
        c->step_ev.push_back(e);
    }
    return SPARC_OK;
}

// flags[F_INPUT_NONFINITE] = 1 when a value of v[0, n) is NaN or infinite.
__global__ __launch_bounds__(256) void k_check_finite(const double* __restrict__ v, long n, int* flags) {
    bool bad = false;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        bad |= !isfinite(v[i]);
    if (__any(bad) && (threadIdx.x & 63) == 0) flags[F_INPUT_NONFINITE] = 1;
}

static sparc_status check_input_density(sparc_gpu_ctx c, const double* rho, long n) {
    k_check_finite<<<(int)std::min<long>(1024, div_up(n, 256)), 256, 0, c->stream>>>(rho, n, c->flags);
    SG_CHECK_LAUNCH(c);
    return SPARC_OK;
}

// Mixing parameters of one SCF iteration (see sparc_gpu_mix).
struct MixArgs {
    double beta, q0;
    int m, period, restart;
    double* hist;
    int iter;
    int nspin;   // 1, or 2 for [rho_up; rho_dn] vectors
};

constexpr int kPulayBlocks = 512;

static size_t mix_red_doubles(int m) {
    return m > 0 ? (size_t)kPulayBlocks * (m * (m + 1) / 2 + m) : 0;
}

// The mixing step, stream-ordered.  Uses fields 0 and 1 as preconditioner
// temporaries (and fields 8, 9 with two spins) and c->red for the Pulay
// partial sums (sized by the caller to mix_red_doubles(m)).
static sparc_status mix_steps(sparc_gpu_ctx c, double* rho_in, const double* rho_out, const MixArgs& a);

static sparc_status mix_impl(sparc_gpu_ctx c, double* rho_in, const double* rho_out, const MixArgs& a) {
    const int slot = prof_begin(c, PK_MIX);
    const sparc_status st = mix_steps(c, rho_in, rho_out, a);
    prof_end(c, slot);
    return st;
}

static sparc_status mix_steps(sparc_gpu_ctx c, double* rho_in, const double* rho_out, const MixArgs& a) {
    const long nd = c->nd;
    const long n = nd * a.nspin;   // length of the mixing vectors
    const int nb = div_up(n, 256);
    const int nb1 = div_up(nd, 256);
    double* t0 = c->field;
    double* t1 = c->field + nd;
    double* fbar = a.nspin == 1 ? t0 : c->field + 8 * nd;
    const bool precond = a.q0 > 0.0;
    bool have_fbar = false;
    if (a.m > 0) {
        const PulayPlan pl = pulay_plan(a.iter, a.m, a.period, a.restart);
        k_pulay_push<<<nb, 256, 0, c->stream>>>(rho_in, rho_out, a.hist, n, a.m, pl.push_slot);
        SG_CHECK_LAUNCH(c);
        if (pl.pulay) {
            SlotList sl{};
            for (int j = 0; j < pl.count; ++j) sl.s[j] = pl.slots[j];
            const int C = pl.count;
            const int nblk = std::min(kPulayBlocks, nb);
            switch (C) {
#define SG_PULAY_DOTS(CC) \
    case CC: k_pulay_dots<CC><<<nblk, 256, 0, c->stream>>>(a.hist, n, a.m, sl, c->red); break;
                SG_PULAY_DOTS(1) SG_PULAY_DOTS(2) SG_PULAY_DOTS(3) SG_PULAY_DOTS(4) SG_PULAY_DOTS(5)
                SG_PULAY_DOTS(6) SG_PULAY_DOTS(7) SG_PULAY_DOTS(8) SG_PULAY_DOTS(9) SG_PULAY_DOTS(10)
#undef SG_PULAY_DOTS
                default: return set_err(c, SPARC_ERR_ARG, "mix: Pulay history too long");
            }
            k_pulay_solve<<<1, 256, 0, c->stream>>>(c->red, nblk, C, c->scal, c->flags);
            k_pulay_apply<<<nb, 256, 0, c->stream>>>(rho_in, a.hist, c->scal, n, a.m, sl, C, a.beta,
                                                     precond ? fbar : nullptr);
            SG_CHECK_LAUNCH(c);
            if (!precond) return SPARC_OK;
            have_fbar = true;
        }
    }
    if (!precond) {
        k_mix_linear<<<nb, 256, 0, c->stream>>>(rho_in, rho_out, a.beta, n);
        SG_CHECK_LAUNCH(c);
        return SPARC_OK;
    }
    // rho_in += beta P r with r = f (or f_bar after a Pulay step), P =
    // (-Lap)(-Lap + q0^2)^-1 in the eigenbasis of the discrete Laplacian;
    // with two spins P acts on r_up + r_dn and r_up - r_dn passes unchanged
    double* diff = c->field + 8 * nd;
    if (a.nspin == 2)
        k_spin_split<<<nb1, 256, 0, c->stream>>>(have_fbar ? fbar : rho_out, have_fbar ? nullptr : rho_in, t0, diff,
                                                 nd);
    else if (!have_fbar)
        k_residual<<<nb1, 256, 0, c->stream>>>(rho_out, rho_in, t0, nd);
    k_axis_transform<<<nb1, 256, 0, c->stream>>>(t0, t1, c->pois_ux, c->nx, c->ny, c->nz, 0, 1);
    k_axis_transform<<<nb1, 256, 0, c->stream>>>(t1, t0, c->pois_uy, c->nx, c->ny, c->nz, 1, 1);
    k_axis_transform<<<nb1, 256, 0, c->stream>>>(t0, t1, c->pois_uz, c->nx, c->ny, c->nz, 2, 1);
    k_kerker<<<nb1, 256, 0, c->stream>>>(t1, c->pois_inv, a.q0 * a.q0, nd);
    k_axis_transform<<<nb1, 256, 0, c->stream>>>(t1, t0, c->pois_uz, c->nx, c->ny, c->nz, 2, 0);
    k_axis_transform<<<nb1, 256, 0, c->stream>>>(t0, t1, c->pois_uy, c->nx, c->ny, c->nz, 1, 0);
    k_axis_transform<<<nb1, 256, 0, c->stream>>>(t1, t0, c->pois_ux, c->nx, c->ny, c->nz, 0, 0);
    if (a.nspin == 2)
        k_spin_combine<<<nb1, 256, 0, c->stream>>>(rho_in, t0, diff, a.beta, nd);
    else
        k_axpy<<<nb1, 256, 0, c->stream>>>(rho_in, t0, a.beta, nd);
    SG_CHECK_LAUNCH(c);
    return SPARC_OK;
}

// Energy terms and residual at (rho_in, rho_out), then the mixing step when
// mix != nullptr, then the copies of the device scalars and flags into the
// context's pinned host mirrors; nothing waits.  Fields: phi = f[2],
// exc = f[3], vxc = f[4]; fields 0, 1 are free.
static sparc_status enqueue_energy(sparc_gpu_ctx c, double* rho_in, const double* rho_out, const MixArgs* mix,
                                   int nspin = 1) {
    const int nblk = std::min(1024, div_up(c->nd, 256));
    sparc_status st = ensure_red(c, std::max((size_t)nblk * kRed, mix ? mix_red_doubles(mix->m) : 0));
    if (st != SPARC_OK) return st;
    const double* phi = c->field + 2 * c->nd;
    const double* exc = c->field + 3 * c->nd;
    const double* vxc = c->field + 4 * c->nd;
    // plain linear mixing is fused into the energy pass (one spin)
    const bool fused = nspin == 1 && mix && mix->m == 0 && !(mix->q0 > 0.0);
    if (nspin == 1)
        k_energy_mix<<<nblk, 256, 0, c->stream>>>(rho_in, rho_out, exc, vxc, phi, c->b, c->nd,
                                                  fused ? mix->beta : 0.0, fused ? 1 : 0, c->red);
    else
        k_energy_spin<<<nblk, 256, 0, c->stream>>>(rho_in, rho_out, exc, vxc, phi, c->b, c->nd, c->red);
    SG_CHECK_LAUNCH(c);
    k_energy_final<<<kRed, 256, 0, c->stream>>>(c->red, nblk, c->scal + S_RED0);
    SG_CHECK_LAUNCH(c);
    if (mix && !fused)
        if ((st = mix_impl(c, rho_in, rho_out, *mix)) != SPARC_OK) return st;
    SG_HIP(c, hipMemcpyAsync(c->h_scal, c->scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    SG_HIP(c, hipMemcpyAsync(c->h_flags, c->flags, F_COUNT * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    return SPARC_OK;
}

// After the call's synchronisation: the device flags raised during the call
// (in this order: non-finite input density, non-SPD Gram matrix, Fermi
// bisection, Pulay normal equations), then the report from the mirrored
// scalars.
static sparc_status read_report(sparc_gpu_ctx c, sparc_gpu_scf_report* rep) {
    const int* fl = c->h_flags;
    const double* h = c->h_scal;
    if (fl[F_INPUT_NONFINITE]) return set_err(c, SPARC_ERR_NONFINITE, "non-finite value in the input density");
    if (fl[F_NOT_SPD]) return set_err(c, SPARC_ERR_NOT_SPD, "Gram matrix of the block is not positive definite");
    if (fl[F_FERMI]) return set_err(c, SPARC_ERR_FERMI, "Fermi level bisection failed");
    if (fl[F_PULAY_SINGULAR]) return set_err(c, SPARC_ERR_SINGULAR, "Pulay normal equations singular");
    const double* r = h + S_RED0;
    const double dV = c->dV;
    sparc_gpu_scf_report R;
    std::memset(&R, 0, sizeof(R));
    R.mu = h[S_OCC];
    R.entropy = h[S_OCC + 1];
    R.band = h[S_OCC + 2];
    R.exc = dV * r[0];
    R.vxc_dc = -dV * r[1];
    R.elec = 0.5 * dV * r[2];
    R.self_energy = -c->e_self;
    R.overlap = c->e_c;
    R.free_energy = R.band + R.exc + R.vxc_dc + R.elec + R.self_energy + R.overlap + R.entropy;
    R.residual = (r[4] > 0.0) ? std::sqrt(r[3] / r[4]) : 0.0;
    if (!std::isfinite(R.free_energy) || !std::isfinite(R.residual))
        return set_err(c, SPARC_ERR_NONFINITE, "non-finite energy or residual");
    if (rep) *rep = R;
    return SPARC_OK;
}

template <typename T>
static sparc_status scf_step_impl(sparc_gpu_ctx c, sparc_gpu_scf_state* s, sparc_gpu_scf_report* rep) {
    sparc_status st;
    const int N = c->n_states;
    T* X = (T*)s->d_X;
    const bool first = s->iter == 0;
    const int npass = first ? s->n_first : 1;
    if ((st = ensure_fields(c, 6)) != SPARC_OK) return st;
    if ((st = ensure_work(c, ((size_t)(N - 1) * s->ldx + c->nd) * sizeof(T))) != SPARC_OK) return st;
    if ((st = ensure_step_events(c, 2 * npass + 6)) != SPARC_OK) return st;
    double* phi = c->field + 2 * c->nd;
    double* exc = c->field + 3 * c->nd;
    double* vxc = c->field + 4 * c->nd;
    double* rho_out = s->d_rho_out ? s->d_rho_out : c->field + 5 * c->nd;
    SG_HIP(c, hipMemsetAsync(c->flags, 0, F_COUNT * sizeof(int), c->stream));
    StepEvents ev(c);
    const int e_begin = ev.mark();
    if ((st = check_input_density(c, s->d_rho_in, c->nd)) != SPARC_OK) return st;
    if ((st = potential_impl(c, s->d_rho_in, phi, exc, vxc, c->veff)) != SPARC_OK) return st;
    if ((st = bounds_impl(c)) != SPARC_OK) return st;
    const int e_pot = ev.mark();
    if (first) {
        if ((st = rayleigh_ritz_impl<T>(c, X, N, s->ldx, s->d_eig, false)) != SPARC_OK) return st;
        k_bounds_from_eig<<<1, 1, 0, c->stream>>>(s->d_eig, N, c->scal, 1);
    } else {
        k_set_ab<<<1, 1, 0, c->stream>>>(c->scal, s->bounds[0], s->bounds[2]);
    }
    SG_CHECK_LAUNCH(c);
    int e_pass[2 * 100 + 1];
    e_pass[0] = ev.mark();
    for (int pass = 0; pass < npass; ++pass) {
        if ((st = filter_impl<T>(c, X, (T*)c->work, N, s->ldx, s->cheb_degree)) != SPARC_OK) return st;
        e_pass[2 * pass + 1] = ev.mark();
        if ((st = rayleigh_ritz_impl<T>(c, X, N, s->ldx, s->d_eig, false)) != SPARC_OK) return st;
        k_bounds_from_eig<<<1, 1, 0, c->stream>>>(s->d_eig, N, c->scal, 0);
        SG_CHECK_LAUNCH(c);
        e_pass[2 * pass + 2] = ev.mark();
    }
    if ((st = occupations_impl(c, s->d_eig, N, s->d_occ, nullptr)) != SPARC_OK) return st;
    if ((st = density_impl<T>(c, X, N, s->ldx, s->d_occ, rho_out)) != SPARC_OK) return st;
    const int e_dens = ev.mark();
    const MixArgs mix{s->mix_beta, s->kerker_q0, s->pulay_history, s->pulay_period, s->pulay_restart, s->d_pulay,
                      s->iter, 1};
    if ((st = enqueue_energy(c, s->d_rho_in, rho_out, &mix)) != SPARC_OK) return st;
    const int e_end = ev.mark();
    SG_HIP(c, hipStreamSynchronize(c->stream));   // the step's one synchronisation
    sparc_gpu_scf_report R;
    if ((st = read_report(c, &R)) != SPARC_OK) return st;
    s->bounds[0] = c->h_scal[S_A];
    s->bounds[1] = c->h_scal[S_B];
    s->bounds[2] = c->h_scal[S_A0];
    double t_filter = 0.0, t_rr = 0.0;
    for (int pass = 0; pass < npass; ++pass) {
        t_filter += ev.ms(e_pass[2 * pass], e_pass[2 * pass + 1]);
        t_rr += ev.ms(e_pass[2 * pass + 1], e_pass[2 * pass + 2]);
    }
    R.t_potential_ms = ev.ms(e_begin, e_pot);
    R.t_filter_ms = t_filter;
    R.t_rr_ms = t_rr;
    R.t_density_ms = ev.ms(e_pass[2 * npass], e_dens);
    R.t_total_ms = ev.ms(e_begin, e_end);
    R.n_passes = npass;
    R.iter = s->iter;
    s->iter += 1;
    if (rep) *rep = R;
    return SPARC_OK;
}

__global__ void k_stash_bounds(double* scal, int spin) {
    scal[S_SPINB + 3 * spin + 0] = scal[S_A];
    scal[S_SPINB + 3 * spin + 1] = scal[S_B];
    scal[S_SPINB + 3 * spin + 2] = scal[S_A0];
}

static sparc_status ensure_veff_spin(sparc_gpu_ctx c) {
    if (c->veff_spin) return SPARC_OK;
    SG_HIP(c, hipMalloc((void**)&c->veff_spin, 2 * (size_t)c->nd * sizeof(double)));
    return SPARC_OK;
}

template <typename T>
static sparc_status scf_step_spin_impl(sparc_gpu_ctx c, sparc_gpu_scf_spin_state* s, sparc_gpu_scf_report* rep) {
    sparc_status st;
    const int N = c->n_states;
    const long nd = c->nd;
    T* Xs[2] = {(T*)s->d_X_up, (T*)s->d_X_dn};
    const bool first = s->iter == 0;
    const int npass = first ? s->n_first : 1;
    if ((st = ensure_fields(c, 10)) != SPARC_OK) return st;
    if ((st = ensure_work(c, ((size_t)(N - 1) * s->ldx + nd) * sizeof(T))) != SPARC_OK) return st;
    if ((st = ensure_veff_spin(c)) != SPARC_OK) return st;
    if ((st = ensure_step_events(c, 2 * (2 * npass + 1) + 6)) != SPARC_OK) return st;
    double* phi = c->field + 2 * nd;
    double* exc = c->field + 3 * nd;
    double* vxc = c->field + 4 * nd;   // 2 N_d
    double* rho_out = s->d_rho_out ? s->d_rho_out : c->field + 6 * nd;
    SG_HIP(c, hipMemsetAsync(c->flags, 0, F_COUNT * sizeof(int), c->stream));
    StepEvents ev(c);
    const int e_begin = ev.mark();
    if ((st = check_input_density(c, s->d_rho_in, 2 * nd)) != SPARC_OK) return st;
    if ((st = potential_spin_impl(c, s->d_rho_in, phi, exc, vxc, c->veff_spin)) != SPARC_OK) return st;
    const int e_pot = ev.mark();
    int e_pass[2][2 * 100 + 1];
    for (int sp = 0; sp < 2; ++sp) {
        T* X = Xs[sp];
        double* eig = s->d_eig + (long)sp * N;
        if ((st = set_veff_impl(c, c->veff_spin + sp * nd)) != SPARC_OK) return st;
        if ((st = bounds_impl(c)) != SPARC_OK) return st;
        if (first) {
            if ((st = rayleigh_ritz_impl<T>(c, X, N, s->ldx, eig, false)) != SPARC_OK) return st;
            k_bounds_from_eig<<<1, 1, 0, c->stream>>>(eig, N, c->scal, 1);
        } else {
            k_set_ab<<<1, 1, 0, c->stream>>>(c->scal, s->bounds[3 * sp], s->bounds[3 * sp + 2]);
        }
        SG_CHECK_LAUNCH(c);
        e_pass[sp][0] = ev.mark();
        for (int pass = 0; pass < npass; ++pass) {
            if ((st = filter_impl<T>(c, X, (T*)c->work, N, s->ldx, s->cheb_degree)) != SPARC_OK) return st;
            e_pass[sp][2 * pass + 1] = ev.mark();
            if ((st = rayleigh_ritz_impl<T>(c, X, N, s->ldx, eig, false)) != SPARC_OK) return st;
            k_bounds_from_eig<<<1, 1, 0, c->stream>>>(eig, N, c->scal, 0);
            SG_CHECK_LAUNCH(c);
            e_pass[sp][2 * pass + 2] = ev.mark();
        }
        k_stash_bounds<<<1, 1, 0, c->stream>>>(c->scal, sp);
        SG_CHECK_LAUNCH(c);
    }
    const int e_dens0 = ev.mark();
    if ((st = occupations_impl(c, s->d_eig, 2 * N, s->d_occ, nullptr, 1.0)) != SPARC_OK) return st;
    for (int sp = 0; sp < 2; ++sp)
        if ((st = density_impl<T>(c, Xs[sp], N, s->ldx, s->d_occ + (long)sp * N, rho_out + sp * nd)) != SPARC_OK)
            return st;
    const int e_dens = ev.mark();
    const MixArgs mix{s->mix_beta, s->kerker_q0, s->pulay_history, s->pulay_period, s->pulay_restart, s->d_pulay,
                      s->iter, 2};
    if ((st = enqueue_energy(c, s->d_rho_in, rho_out, &mix, 2)) != SPARC_OK) return st;
    const int e_end = ev.mark();
    SG_HIP(c, hipStreamSynchronize(c->stream));   // the step's one synchronisation
    sparc_gpu_scf_report R;
    if ((st = read_report(c, &R)) != SPARC_OK) return st;
    for (int k = 0; k < 6; ++k) s->bounds[k] = c->h_scal[S_SPINB + k];
    double t_filter = 0.0, t_rr = 0.0;
    for (int sp = 0; sp < 2; ++sp)
        for (int pass = 0; pass < npass; ++pass) {
            t_filter += ev.ms(e_pass[sp][2 * pass], e_pass[sp][2 * pass + 1]);
            t_rr += ev.ms(e_pass[sp][2 * pass + 1], e_pass[sp][2 * pass + 2]);
        }
    R.t_potential_ms = ev.ms(e_begin, e_pot);
    R.t_filter_ms = t_filter;
    R.t_rr_ms = t_rr;
    R.t_density_ms = ev.ms(e_dens0, e_dens);
    R.t_total_ms = ev.ms(e_begin, e_end);
    R.n_passes = 2 * npass;
    R.iter = s->iter;
    s->iter += 1;
    if (rep) *rep = R;
    return SPARC_OK;
}

static bool ranges_overlap(const void* a, const void* b, size_t bytes) {
    const char* pa = (const char*)a;
    const char* pb = (const char*)b;
    return pa < pb + bytes && pb < pa + bytes;
}

static sparc_status check_spin_state(sparc_gpu_ctx c, const sparc_gpu_scf_spin_state* s) {
    if (!s) return set_err(c, SPARC_ERR_ARG, "scf_spin: null state");
    if (!s->d_rho_in || !s->d_X_up || !s->d_X_dn || !s->d_eig || !s->d_occ)
        return set_err(c, SPARC_ERR_ARG, "scf_spin: null buffer");
    if (s->prec != SPARC_FP64 && s->prec != SPARC_FP32) return set_err(c, SPARC_ERR_ARG, "scf_spin: bad precision");
    if (s->ldx < c->nd) return set_err(c, SPARC_ERR_ARG, "scf_spin: ldx < N_d");
    const size_t es = s->prec == SPARC_FP64 ? 8 : 4;
    if (ranges_overlap(s->d_X_up, s->d_X_dn, ((size_t)(c->n_states - 1) * s->ldx + c->nd) * es))
        return set_err(c, SPARC_ERR_ARG, "scf_spin: the two spin blocks overlap");
    if (s->cheb_degree < 1 || s->cheb_degree > 10000) return set_err(c, SPARC_ERR_ARG, "scf_spin: bad degree");
    if (s->n_first < 1 || s->n_first > 100) return set_err(c, SPARC_ERR_ARG, "scf_spin: bad n_first");
    if (!(s->mix_beta > 0.0 && s->mix_beta <= 1.0)) return set_err(c, SPARC_ERR_ARG, "scf_spin: bad mix_beta");
    if (!(s->kerker_q0 >= 0.0) || !std::isfinite(s->kerker_q0))
        return set_err(c, SPARC_ERR_ARG, "scf_spin: bad kerker_q0");
    if (s->pulay_history < 0 || s->pulay_history > SPARC_PULAY_MAX)
        return set_err(c, SPARC_ERR_ARG, "scf_spin: pulay_history outside [0, SPARC_PULAY_MAX]");
    if (s->pulay_history > 0 && (s->pulay_period < 1 || (s->pulay_restart != 0 && s->pulay_restart != 1) ||
                                 !s->d_pulay))
        return set_err(c, SPARC_ERR_ARG, "scf_spin: bad Pulay period, restart flag or history buffer");
    if (s->iter < 0) return set_err(c, SPARC_ERR_ARG, "scf_spin: negative iter");
    if (s->iter > 0 && !(s->bounds[2] < s->bounds[0] && s->bounds[5] < s->bounds[3]))
        return set_err(c, SPARC_ERR_ARG, "scf_spin: bounds need a0 < a after the first iteration");
    return SPARC_OK;
}

// ---- Bloch k-points ---------------------------------------------------------

// rho (+)= w_k sum_j occ_j (u_j^2 + v_j^2) over Bloch columns [u; v]
template <typename T>
__global__ __launch_bounds__(256) void k_density_k(const T* __restrict__ X, int ncol, long ldx, long nd,
                                                   const double* __restrict__ occ, double wk,
                                                   double* __restrict__ rho, int accumulate) {
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nd) return;
    double acc = 0.0;
    for (int j = 0; j < ncol; ++j) {
        const double u = (double)X[p + (long)j * ldx], v = (double)X[nd + p + (long)j * ldx];
        acc += occ[j] * (u * u + v * v);
    }
    rho[p] = (accumulate ? rho[p] : 0.0) + wk * acc;
}

__global__ void k_stash_kbounds(const double* scal, double* dst, int q) {
    dst[3 * q + 0] = scal[S_A];
    dst[3 * q + 1] = scal[S_B];
    dst[3 * q + 2] = scal[S_A0];
}

static sparc_status ensure_dev(sparc_gpu_ctx c, double** p, int* have, int need) {
    if (*have >= need) return SPARC_OK;
    if (*p) {
        SG_HIP(c, hipStreamSynchronize(c->stream));
        SG_HIP(c, hipFree(*p));
        *p = nullptr;
        *have = 0;
    }
    SG_HIP(c, hipMalloc((void**)p, (size_t)need * sizeof(double)));
    *have = need;
    return SPARC_OK;
}

template <typename T>
static sparc_status scf_step_k_impl(sparc_gpu_ctx c, sparc_gpu_scf_k_state* s, sparc_gpu_scf_report* rep) {
    sparc_status st;
    const int N2 = 2 * c->n_states;
    const int nk = s->n_k;
    const long nd = c->nd;
    if ((st = ensure_fields(c, 6)) != SPARC_OK) return st;
    if ((st = ensure_work(c, ((size_t)(N2 - 1) * s->ldx + 2 * nd) * sizeof(T))) != SPARC_OK) return st;
    if ((st = ensure_dev(c, &c->kp_bounds, &c->kp_bounds_n, 3 * nk)) != SPARC_OK) return st;
    if ((st = ensure_dev(c, &c->kp_wts, &c->kp_wts_n, nk * N2)) != SPARC_OK) return st;
    {
        std::vector<double> w((size_t)nk * N2);
        for (int q = 0; q < nk; ++q)
            for (int j = 0; j < N2; ++j) w[(size_t)q * N2 + j] = s->kweights[q];
        SG_HIP(c, hipMemcpy(c->kp_wts, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    if ((st = ensure_step_events(c, nk * (2 * s->n_first + 1) + 6)) != SPARC_OK) return st;
    double* phi = c->field + 2 * nd;
    double* exc = c->field + 3 * nd;
    double* vxc = c->field + 4 * nd;
    double* rho_out = s->d_rho_out ? s->d_rho_out : c->field + 5 * nd;
    SG_HIP(c, hipMemsetAsync(c->flags, 0, F_COUNT * sizeof(int), c->stream));
    StepEvents ev(c);
    const int e_begin = ev.mark();
    if ((st = check_input_density(c, s->d_rho_in, nd)) != SPARC_OK) return st;
    if ((st = potential_impl(c, s->d_rho_in, phi, exc, vxc, c->veff)) != SPARC_OK) return st;
    const int e_pot = ev.mark();
    const bool first = s->iter == 0;
    const int npass = first ? s->n_first : 1;
    std::vector<int> e_pass;   // per k: start, then (filter end, RR end) per pass
    for (int q = 0; q < nk; ++q) {
        for (int d = 0; d < 3; ++d) c->kvec[d] = s->kpts[3 * q + d];
        T* X = (T*)s->d_X[q];
        double* eig = s->d_eig + (long)q * N2;
        if ((st = bloch_bounds_impl(c)) != SPARC_OK) return st;
        if (first) {
            if ((st = rayleigh_ritz_k_impl<T>(c, X, N2, s->ldx, eig, false)) != SPARC_OK) return st;
            k_bounds_from_eig<<<1, 1, 0, c->stream>>>(eig, N2, c->scal, 1);
        } else {
            k_set_ab<<<1, 1, 0, c->stream>>>(c->scal, s->bounds[3 * q], s->bounds[3 * q + 2]);
        }
        SG_CHECK_LAUNCH(c);
        e_pass.push_back(ev.mark());
        for (int pass = 0; pass < npass; ++pass) {
            if ((st = bloch_filter_impl<T>(c, X, (T*)c->work, N2, s->ldx, s->cheb_degree)) != SPARC_OK) return st;
            e_pass.push_back(ev.mark());
            if ((st = rayleigh_ritz_k_impl<T>(c, X, N2, s->ldx, eig, false)) != SPARC_OK) return st;
            k_bounds_from_eig<<<1, 1, 0, c->stream>>>(eig, N2, c->scal, 0);
            SG_CHECK_LAUNCH(c);
            e_pass.push_back(ev.mark());
        }
        k_stash_kbounds<<<1, 1, 0, c->stream>>>(c->scal, c->kp_bounds, q);
        SG_CHECK_LAUNCH(c);
    }
    const int e_dens0 = ev.mark();
    if ((st = occupations_impl(c, s->d_eig, nk * N2, s->d_occ, nullptr, 1.0, c->kp_wts)) != SPARC_OK) return st;
    for (int q = 0; q < nk; ++q) {
        k_density_k<T><<<div_up(nd, 256), 256, 0, c->stream>>>((const T*)s->d_X[q], N2, s->ldx, nd,
                                                               s->d_occ + (long)q * N2, s->kweights[q], rho_out,
                                                               q > 0 ? 1 : 0);
        SG_CHECK_LAUNCH(c);
    }
    const int e_dens = ev.mark();
    const MixArgs mix{s->mix_beta, s->kerker_q0, s->pulay_history, s->pulay_period, s->pulay_restart, s->d_pulay,
                      s->iter, 1};
    if ((st = enqueue_energy(c, s->d_rho_in, rho_out, &mix)) != SPARC_OK) return st;
    const int e_end = ev.mark();
    SG_HIP(c, hipStreamSynchronize(c->stream));
    sparc_gpu_scf_report R;
    if ((st = read_report(c, &R)) != SPARC_OK) return st;
    SG_HIP(c, hipMemcpy(s->bounds, c->kp_bounds, 3 * (size_t)nk * sizeof(double), hipMemcpyDeviceToHost));
    double t_filter = 0.0, t_rr = 0.0;
    for (int q = 0; q < nk; ++q) {
        const int* e = e_pass.data() + (size_t)q * (2 * npass + 1);
        for (int pass = 0; pass < npass; ++pass) {
            t_filter += ev.ms(e[2 * pass], e[2 * pass + 1]);
            t_rr += ev.ms(e[2 * pass + 1], e[2 * pass + 2]);
        }
    }
    R.t_potential_ms = ev.ms(e_begin, e_pot);
    R.t_filter_ms = t_filter;
    R.t_rr_ms = t_rr;
    R.t_density_ms = ev.ms(e_dens0, e_dens);
    R.t_total_ms = ev.ms(e_begin, e_end);
    R.n_passes = nk * npass;
    R.iter = s->iter;
    s->iter += 1;
    if (rep) *rep = R;
    return SPARC_OK;
}

static sparc_status check_k_state(sparc_gpu_ctx c, const sparc_gpu_scf_k_state* s) {
    if (!s) return set_err(c, SPARC_ERR_ARG, "scf_k: null state");
    if (s->n_k < 1 || s->n_k > 4096) return set_err(c, SPARC_ERR_ARG, "scf_k: n_k outside [1, 4096]");
    if (!s->kpts || !s->kweights || !s->d_X || !s->bounds) return set_err(c, SPARC_ERR_ARG, "scf_k: null host array");
    double wsum = 0.0;
    for (int q = 0; q < s->n_k; ++q) {
        if (!s->d_X[q]) return set_err(c, SPARC_ERR_ARG, "scf_k: null orbital block");
        if (!(s->kweights[q] > 0.0) || !std::isfinite(s->kweights[q]))
            return set_err(c, SPARC_ERR_ARG, "scf_k: k weights must be positive");
        for (int d = 0; d < 3; ++d)
            if (!std::isfinite(s->kpts[3 * q + d])) return set_err(c, SPARC_ERR_ARG, "scf_k: non-finite k");
        wsum += s->kweights[q];
    }
    if (std::fabs(wsum - 1.0) > 1e-12) return set_err(c, SPARC_ERR_ARG, "scf_k: k weights must sum to 1");
    if (!s->d_rho_in || !s->d_eig || !s->d_occ) return set_err(c, SPARC_ERR_ARG, "scf_k: null buffer");
    if (s->prec != SPARC_FP64 && s->prec != SPARC_FP32) return set_err(c, SPARC_ERR_ARG, "scf_k: bad precision");
    if (s->ldx < 2 * c->nd) return set_err(c, SPARC_ERR_ARG, "scf_k: ldx < 2 N_d");
    if (2 * c->n_states > kEighMaxN) return set_err(c, SPARC_ERR_ARG, "scf_k: 2 n_states above the eigensolver limit");
    if (s->cheb_degree < 1 || s->cheb_degree > 10000) return set_err(c, SPARC_ERR_ARG, "scf_k: bad degree");
    if (s->n_first < 1 || s->n_first > 100) return set_err(c, SPARC_ERR_ARG, "scf_k: bad n_first");
    if (!(s->mix_beta > 0.0 && s->mix_beta <= 1.0)) return set_err(c, SPARC_ERR_ARG, "scf_k: bad mix_beta");
    if (!(s->kerker_q0 >= 0.0) || !std::isfinite(s->kerker_q0)) return set_err(c, SPARC_ERR_ARG, "scf_k: bad kerker_q0");
    if (s->pulay_history < 0 || s->pulay_history > SPARC_PULAY_MAX)
        return set_err(c, SPARC_ERR_ARG, "scf_k: pulay_history outside [0, SPARC_PULAY_MAX]");
    if (s->pulay_history > 0 && (s->pulay_period < 1 || (s->pulay_restart != 0 && s->pulay_restart != 1) ||
                                 !s->d_pulay))
        return set_err(c, SPARC_ERR_ARG, "scf_k: bad Pulay period, restart flag or history buffer");
    if (s->iter < 0) return set_err(c, SPARC_ERR_ARG, "scf_k: negative iter");
    if (s->iter > 0)
        for (int q = 0; q < s->n_k; ++q)
            if (!(s->bounds[3 * q + 2] < s->bounds[3 * q]))
                return set_err(c, SPARC_ERR_ARG, "scf_k: bounds need a0 < a after the first iteration");
    return SPARC_OK;
}

static sparc_status check_state(sparc_gpu_ctx c, const sparc_gpu_scf_state* s) {
    if (!s) return set_err(c, SPARC_ERR_ARG, "scf: null state");
    if (!s->d_rho_in || !s->d_X || !s->d_eig || !s->d_occ) return set_err(c, SPARC_ERR_ARG, "scf: null buffer");
    if (s->prec != SPARC_FP64 && s->prec != SPARC_FP32) return set_err(c, SPARC_ERR_ARG, "scf: bad precision");
    if (s->ldx < c->nd) return set_err(c, SPARC_ERR_ARG, "scf: ldx < N_d");
    if (s->cheb_degree < 1 || s->cheb_degree > 10000) return set_err(c, SPARC_ERR_ARG, "scf: bad degree");
    if (s->n_first < 1 || s->n_first > 100) return set_err(c, SPARC_ERR_ARG, "scf: bad n_first");
    if (!(s->mix_beta > 0.0 && s->mix_beta <= 1.0)) return set_err(c, SPARC_ERR_ARG, "scf: bad mix_beta");
    if (!(s->kerker_q0 >= 0.0) || !std::isfinite(s->kerker_q0)) return set_err(c, SPARC_ERR_ARG, "scf: bad kerker_q0");
    if (s->pulay_history < 0 || s->pulay_history > SPARC_PULAY_MAX)
        return set_err(c, SPARC_ERR_ARG, "scf: pulay_history outside [0, SPARC_PULAY_MAX]");
    if (s->pulay_history > 0 && (s->pulay_period < 1 || (s->pulay_restart != 0 && s->pulay_restart != 1) ||
                                 !s->d_pulay))
        return set_err(c, SPARC_ERR_ARG, "scf: bad Pulay period, restart flag or history buffer");
    if (s->iter < 0) return set_err(c, SPARC_ERR_ARG, "scf: negative iter");
    if (s->iter > 0 && !(s->bounds[2] < s->bounds[0]))
        return set_err(c, SPARC_ERR_ARG, "scf: bounds need a0 < a after the first iteration");
    return SPARC_OK;
}

}  // namespace sg

using namespace sg;

extern "C" {

sparc_status sparc_gpu_scf_step(sparc_gpu_ctx c, sparc_gpu_scf_state* s, sparc_gpu_scf_report* rep) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    sparc_status st = check_state(c, s);
    if (st != SPARC_OK) return st;
    if (s->prec == SPARC_FP64) return scf_step_impl<double>(c, s, rep);
    return scf_step_impl<float>(c, s, rep);
}

sparc_status sparc_gpu_final_rr_fp64(sparc_gpu_ctx c, sparc_gpu_scf_state* s, double* d_X64, long ldx64,
                                     sparc_gpu_scf_report* rep) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    sparc_status st = check_state(c, s);
    if (st != SPARC_OK) return st;
    if (!d_X64 || ldx64 < c->nd) return set_err(c, SPARC_ERR_ARG, "final_rr_fp64: bad FP64 block");
    const int N = c->n_states;
    if ((st = ensure_fields(c, 6)) != SPARC_OK) return st;
    if ((st = ensure_step_events(c, 5)) != SPARC_OK) return st;
    StepEvents ev(c);
    const int e_begin = ev.mark();   // the promotion of the block is part of the call's time
    dim3 grid(div_up(c->nd, 256), N);
    if (s->prec == SPARC_FP32)
        k_promote<float><<<grid, 256, 0, c->stream>>>((const float*)s->d_X, d_X64, c->nd, N, s->ldx, ldx64);
    else
        k_promote<double><<<grid, 256, 0, c->stream>>>((const double*)s->d_X, d_X64, c->nd, N, s->ldx, ldx64);
    SG_CHECK_LAUNCH(c);
    SG_HIP(c, hipMemsetAsync(c->flags, 0, F_COUNT * sizeof(int), c->stream));
    double* phi = c->field + 2 * c->nd;
    double* exc = c->field + 3 * c->nd;
    double* vxc = c->field + 4 * c->nd;
    double* rho_out = s->d_rho_out ? s->d_rho_out : c->field + 5 * c->nd;
    if ((st = check_input_density(c, s->d_rho_in, c->nd)) != SPARC_OK) return st;
    if ((st = potential_impl(c, s->d_rho_in, phi, exc, vxc, c->veff)) != SPARC_OK) return st;
    const int e_pot = ev.mark();
    if ((st = rayleigh_ritz_impl<double>(c, d_X64, N, ldx64, s->d_eig, false)) != SPARC_OK) return st;
    const int e_rr = ev.mark();
    if ((st = occupations_impl(c, s->d_eig, N, s->d_occ, nullptr)) != SPARC_OK) return st;
    if ((st = density_impl<double>(c, d_X64, N, ldx64, s->d_occ, rho_out)) != SPARC_OK) return st;
    const int e_dens = ev.mark();
    if ((st = enqueue_energy(c, s->d_rho_in, rho_out, nullptr)) != SPARC_OK) return st;
    const int e_end = ev.mark();
    SG_HIP(c, hipStreamSynchronize(c->stream));   // the call's one synchronisation
    sparc_gpu_scf_report R;
    if ((st = read_report(c, &R)) != SPARC_OK) return st;
    R.t_potential_ms = ev.ms(e_begin, e_pot);
    R.t_rr_ms = ev.ms(e_pot, e_rr);
    R.t_density_ms = ev.ms(e_rr, e_dens);
    R.t_total_ms = ev.ms(e_begin, e_end);
    R.n_passes = 0;
    R.iter = s->iter;
    if (rep) *rep = R;
    return SPARC_OK;
}

sparc_status sparc_gpu_density(sparc_gpu_ctx c, sparc_prec prec, const void* d_X, int ncol, long ldx,
                               const double* d_occ, double* d_rho) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    if (prec != SPARC_FP64 && prec != SPARC_FP32) return set_err(c, SPARC_ERR_ARG, "density: bad precision");
    if (!d_X || !d_occ || !d_rho) return set_err(c, SPARC_ERR_ARG, "density: null pointer");
    if (ncol < 1 || ncol > c->n_states) return set_err(c, SPARC_ERR_ARG, "density: ncol out of range");
    if (ldx < c->nd) return set_err(c, SPARC_ERR_ARG, "density: ldx < N_d");
    if (prec == SPARC_FP64) return density_impl<double>(c, (const double*)d_X, ncol, ldx, d_occ, d_rho);
    return density_impl<float>(c, (const float*)d_X, ncol, ldx, d_occ, d_rho);
}

sparc_status sparc_gpu_mix(sparc_gpu_ctx c, double* d_rho_in, const double* d_rho_out, int n_spin, double beta,
                           double kerker_q0, int pulay_history, int pulay_period, int restart, double* d_hist,
                           int iter) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    if (!d_rho_in || !d_rho_out) return set_err(c, SPARC_ERR_ARG, "mix: null density");
    if (n_spin != 1 && n_spin != 2) return set_err(c, SPARC_ERR_ARG, "mix: n_spin must be 1 or 2");
    if (!(beta > 0.0 && beta <= 1.0)) return set_err(c, SPARC_ERR_ARG, "mix: bad beta");
    if (!(kerker_q0 >= 0.0) || !std::isfinite(kerker_q0)) return set_err(c, SPARC_ERR_ARG, "mix: bad kerker_q0");
    if (pulay_history < 0 || pulay_history > SPARC_PULAY_MAX)
        return set_err(c, SPARC_ERR_ARG, "mix: pulay_history outside [0, SPARC_PULAY_MAX]");
    if (pulay_history > 0 && (pulay_period < 1 || (restart != 0 && restart != 1) || !d_hist))
        return set_err(c, SPARC_ERR_ARG, "mix: bad Pulay period, restart flag or history buffer");
    if (iter < 0) return set_err(c, SPARC_ERR_ARG, "mix: negative iter");
    sparc_status st;
    if ((st = ensure_fields(c, n_spin == 2 ? 10 : 2)) != SPARC_OK) return st;
    if ((st = ensure_red(c, mix_red_doubles(pulay_history))) != SPARC_OK) return st;
    SG_HIP(c, hipMemsetAsync(c->flags + F_PULAY_SINGULAR, 0, sizeof(int), c->stream));
    const MixArgs mix{beta, kerker_q0, pulay_history, pulay_period, restart, d_hist, iter, n_spin};
    if ((st = mix_impl(c, d_rho_in, d_rho_out, mix)) != SPARC_OK) return st;
    int flag = 0;
    SG_HIP(c, hipMemcpyAsync(&flag, c->flags + F_PULAY_SINGULAR, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    SG_HIP(c, hipStreamSynchronize(c->stream));
    if (flag) return set_err(c, SPARC_ERR_SINGULAR, "Pulay normal equations singular");
    return SPARC_OK;
}

sparc_status sparc_gpu_scf_step_spin(sparc_gpu_ctx c, sparc_gpu_scf_spin_state* s, sparc_gpu_scf_report* rep) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    sparc_status st = check_spin_state(c, s);
    if (st != SPARC_OK) return st;
    if (s->prec == SPARC_FP64) return scf_step_spin_impl<double>(c, s, rep);
    return scf_step_spin_impl<float>(c, s, rep);
}

sparc_status sparc_gpu_scf_step_k(sparc_gpu_ctx c, sparc_gpu_scf_k_state* s, sparc_gpu_scf_report* rep) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    sparc_status st = check_k_state(c, s);
    if (st != SPARC_OK) return st;
    if (s->prec == SPARC_FP64) return scf_step_k_impl<double>(c, s, rep);
    return scf_step_k_impl<float>(c, s, rep);
}

sparc_status sparc_gpu_potential_spin(sparc_gpu_ctx c, const double* d_rho, double* d_phi, double* d_exc,
                                      double* d_vxc, double* d_veff) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    if (!d_rho) return set_err(c, SPARC_ERR_ARG, "potential_spin: null density");
    return potential_spin_impl(c, d_rho, d_phi, d_exc, d_vxc, d_veff);
}

sparc_status sparc_gpu_occupations_spin(sparc_gpu_ctx c, const double* d_eig, int ncol, double* d_occ,
                                        double* d_mu) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    if (!d_eig || !d_occ) return set_err(c, SPARC_ERR_ARG, "occupations_spin: null pointer");
    if (ncol < 1 || ncol > c->n_states) return set_err(c, SPARC_ERR_ARG, "occupations_spin: ncol out of range");
    if (c->n_electrons > 2.0 * ncol) return set_err(c, SPARC_ERR_ARG, "occupations_spin: N_e > 2 ncol");
    return occupations_impl(c, d_eig, 2 * ncol, d_occ, d_mu, 1.0);
}

sparc_status sparc_gpu_occupations(sparc_gpu_ctx c, const double* d_eig, int ncol, double* d_occ, double* d_mu) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    if (!d_eig || !d_occ) return set_err(c, SPARC_ERR_ARG, "occupations: null pointer");
    if (ncol < 1 || ncol > c->n_states) return set_err(c, SPARC_ERR_ARG, "occupations: ncol out of range");
    if (c->n_electrons > 2.0 * ncol) return set_err(c, SPARC_ERR_ARG, "occupations: N_e > 2 ncol");
    return occupations_impl(c, d_eig, ncol, d_occ, d_mu);
}

sparc_status sparc_gpu_potential(sparc_gpu_ctx c, const double* d_rho, double* d_phi, double* d_exc, double* d_vxc,
                                 double* d_veff) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    if (!d_rho) return set_err(c, SPARC_ERR_ARG, "potential: null density");
    if (d_veff == c->veff) return set_err(c, SPARC_ERR_ARG, "potential: output aliases the context");
    return potential_impl(c, d_rho, d_phi, d_exc, d_vxc, d_veff);
}

}  // extern "C"
