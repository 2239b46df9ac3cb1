// Context creation, geometry tables and small public entry points.
//
// Geometry set-up (Sec. 2.1): uniform periodic grid, centred finite
// differences, local real-space electrostatics with Gaussian pseudocharges,
// and Kleinman-Bylander projector tables for the outer-product nonlocal
// operator.  The host only enumerates which grid points (and periodic images)
// fall inside each atom's cut-off; every field value is evaluated on the GPU.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <numeric>
#include <unordered_map>

#include "internal.hpp"

namespace sg {

sparc_status set_err(sparc_gpu_ctx c, sparc_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

sparc_status hip_err(sparc_gpu_ctx c, hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory) return set_err(c, SPARC_ERR_NOMEM, m);
    return set_err(c, SPARC_ERR_HIP, m);
}

static sparc_status grow(sparc_gpu_ctx c, void** p, size_t* have, size_t need) {
    if (*have >= need) return SPARC_OK;
    if (*p) {
        SG_HIP(c, hipStreamSynchronize(c->stream));
        SG_HIP(c, hipFree(*p));
        *p = nullptr;
        *have = 0;
    }
    SG_HIP(c, hipMalloc(p, need));
    *have = need;
    return SPARC_OK;
}

sparc_status ensure_work(sparc_gpu_ctx c, size_t bytes) { return grow(c, &c->work, &c->work_bytes, bytes); }

int prof_begin(sparc_gpu_ctx c, int kernel, hipStream_t s) {
    if (!c->prof) return -1;
    int slot = c->prof_used;
    if (2 * (size_t)(slot + 1) > c->prof_pool.size()) {
        for (int i = 0; i < 2; ++i) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return -1;
            c->prof_pool.push_back(e);
        }
        c->prof_kernel.push_back(0);
    }
    c->prof_kernel[slot] = kernel;
    c->prof_used++;
    hipEventRecord(c->prof_pool[2 * slot], s ? s : c->stream);
    return slot;
}

void prof_end(sparc_gpu_ctx c, int slot, hipStream_t s) {
    if (slot < 0) return;
    hipEventRecord(c->prof_pool[2 * slot + 1], s ? s : c->stream);
}

static sparc_status prof_flush(sparc_gpu_ctx c) {
    if (c->prof_used == 0) return SPARC_OK;
    SG_HIP(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < c->prof_used; ++i) {
        float ms = 0.f;
        SG_HIP(c, hipEventElapsedTime(&ms, c->prof_pool[2 * i], c->prof_pool[2 * i + 1]));
        c->prof_ms[c->prof_kernel[i]] += ms;
        c->prof_n[c->prof_kernel[i]] += 1;
    }
    c->prof_used = 0;
    return SPARC_OK;
}

sparc_status ensure_gemm_part(sparc_gpu_ctx c, size_t elems) {
    size_t have = c->gemm_part_elems * sizeof(double);
    sparc_status s = grow(c, (void**)&c->gemm_part, &have, elems * sizeof(double));
    c->gemm_part_elems = have / sizeof(double);
    return s;
}

sparc_status ensure_small(sparc_gpu_ctx c, size_t elems) {
    size_t have = c->small_elems * sizeof(double);
    sparc_status s = grow(c, (void**)&c->small, &have, elems * sizeof(double));
    c->small_elems = have / sizeof(double);
    return s;
}

sparc_status ensure_red(sparc_gpu_ctx c, size_t elems) {
    size_t have = c->red_elems * sizeof(double);
    sparc_status s = grow(c, (void**)&c->red, &have, elems * sizeof(double));
    c->red_elems = have / sizeof(double);
    return s;
}

sparc_status ensure_fields(sparc_gpu_ctx c, int n) {
    if (c->n_field >= n) return SPARC_OK;
    size_t have = (size_t)c->n_field * c->nd * sizeof(double);
    sparc_status s = grow(c, (void**)&c->field, &have, (size_t)n * c->nd * sizeof(double));
    if (s == SPARC_OK) c->n_field = n;
    return s;
}

// ------------------------------------------------------------------ kernels

// b(p) = -sum_I sum_images Z_I (pi rc_I^2)^-3/2 exp(-d^2/rc_I^2), d <= rmax_I
// (or the analogous positive atomic densities when sign > 0).
struct AtomImages {
    double x, y, z;     // position
    double amp;         // prefactor of the Gaussian
    double inv_w2;      // 1 / width^2
    double rmax2;       // squared cut-off
    int n0[3], n1[3];   // image shift ranges per axis
};

__global__ void k_gaussian_field(const AtomImages* at, int n_atoms, int nx, int ny, int nz, double hx,
                                 double hy, double hz, double Lx, double Ly, double Lz, double* out) {
    long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long nd = (long)nx * ny * nz;
    if (p >= nd) return;
    int ix = (int)(p % nx);
    int iy = (int)((p / nx) % ny);
    int iz = (int)(p / ((long)nx * ny));
    double px = ix * hx, py = iy * hy, pz = iz * hz;
    double acc = 0.0;
    for (int a = 0; a < n_atoms; ++a) {
        AtomImages A = at[a];
        for (int kz = A.n0[2]; kz <= A.n1[2]; ++kz) {
            double dz = pz - A.z - kz * Lz;
            for (int ky = A.n0[1]; ky <= A.n1[1]; ++ky) {
                double dy = py - A.y - ky * Ly;
                for (int kx = A.n0[0]; kx <= A.n1[0]; ++kx) {
                    double dx = px - A.x - kx * Lx;
                    double r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 <= A.rmax2) acc += A.amp * exp(-r2 * A.inv_w2);
                }
            }
        }
    }
    out[p] = acc;
}

// One block per atom: 1/2 dV sum over its (unwrapped) ball of b_I V_I, with
// V_I(r) = -Z erf(r/rc)/r and its r -> 0 limit.  Partial per atom.
__global__ void k_self_energy(const AtomImages* at, const double* Zs, const double* rcs, int n_atoms, double hx,
                              double hy, double hz, double dV, double* part) {
    int a = blockIdx.x;
    AtomImages A = at[a];
    double Z = Zs[a], rc = rcs[a];
    double rmax = sqrt(A.rmax2);
    int lo[3], hi[3];
    double c[3] = {A.x, A.y, A.z}, h[3] = {hx, hy, hz};
    for (int d = 0; d < 3; ++d) {
        lo[d] = (int)ceil((c[d] - rmax) / h[d]);
        hi[d] = (int)floor((c[d] + rmax) / h[d]);
    }
    int nxb = hi[0] - lo[0] + 1, nyb = hi[1] - lo[1] + 1, nzb = hi[2] - lo[2] + 1;
    long tot = (long)nxb * nyb * nzb;
    double acc = 0.0;
    const double pi = 3.14159265358979323846;
    for (long t = threadIdx.x; t < tot; t += blockDim.x) {
        int i = lo[0] + (int)(t % nxb);
        int j = lo[1] + (int)((t / nxb) % nyb);
        int k = lo[2] + (int)(t / ((long)nxb * nyb));
        double dx = i * hx - A.x, dy = j * hy - A.y, dz = k * hz - A.z;
        double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 > A.rmax2) continue;
        double bI = A.amp * exp(-r2 * A.inv_w2);
        double r = sqrt(r2);
        double V = (r < 1e-12) ? -2.0 * Z / (sqrt(pi) * rc) : -Z * erf(r / rc) / r;
        acc += bI * V;
    }
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[a] = 0.5 * dV * red[0];
}

// Overlap correction: thread per ordered pair (I, J), images with d < rmax.
__global__ void k_overlap(const double* pos, const double* Z, const double* rc, int n_atoms, double Lx, double Ly,
                          double Lz, double rmax, int nimx, int nimy, int nimz, double* part) {
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)n_atoms * n_atoms) return;
    int I = (int)(t / n_atoms), J = (int)(t % n_atoms);
    double s = sqrt(rc[I] * rc[I] + rc[J] * rc[J]);
    double acc = 0.0;
    for (int a = -nimx; a <= nimx; ++a)
        for (int b = -nimy; b <= nimy; ++b)
            for (int cc = -nimz; cc <= nimz; ++cc) {
                if (I == J && a == 0 && b == 0 && cc == 0) continue;
                double dx = pos[3 * J] + a * Lx - pos[3 * I];
                double dy = pos[3 * J + 1] + b * Ly - pos[3 * I + 1];
                double dz = pos[3 * J + 2] + cc * Lz - pos[3 * I + 2];
                double d = sqrt(dx * dx + dy * dy + dz * dz);
                if (d < rmax) acc += 0.5 * Z[I] * Z[J] * erfc(d / s) / d;
            }
    part[t] = acc;
}

// Fixed-order sum of n values by one block (deterministic).
__global__ void k_sum_serial(const double* v, long n, double* out) {
    __shared__ double red[256];
    double acc = 0.0;
    for (long i = threadIdx.x; i < n; i += blockDim.x) acc += v[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// Projector values on each unique support point: sum over its periodic images
// of chi_s = N0 e, chi_p = N1 {dx,dy,dz} e, e = exp(-r^2/rc^2).
__global__ void k_projector_values(const int* img_off, const int* img_ijk, const int* sup_atom, const double* pos,
                                   long n_sup, double hx, double hy, double hz, double inv_rc2, double N0, double N1,
                                   double* chi) {
    long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_sup) return;
    int a = sup_atom[s];
    double ax = pos[3 * a], ay = pos[3 * a + 1], az = pos[3 * a + 2];
    double v0 = 0, v1 = 0, v2 = 0, v3 = 0;
    for (int e = img_off[s]; e < img_off[s + 1]; ++e) {
        double dx = img_ijk[3 * e] * hx - ax;
        double dy = img_ijk[3 * e + 1] * hy - ay;
        double dz = img_ijk[3 * e + 2] * hz - az;
        double ex = exp(-(dx * dx + dy * dy + dz * dz) * inv_rc2);
        v0 += N0 * ex;
        v1 += N1 * dx * ex;
        v2 += N1 * dy * ex;
        v3 += N1 * dz * ex;
    }
    chi[4 * s + 0] = v0;
    chi[4 * s + 1] = v1;
    chi[4 * s + 2] = v2;
    chi[4 * s + 3] = v3;
}

// dV ||chi_lm||^2 per atom (one block per atom).
__global__ void k_projector_norms(const long* sup_off, const double* chi, double dV, double* norms) {
    int a = blockIdx.x;
    __shared__ double red[4][256];
    double acc[4] = {0, 0, 0, 0};
    for (long s = sup_off[a] + threadIdx.x; s < sup_off[a + 1]; s += blockDim.x)
        for (int k = 0; k < 4; ++k) acc[k] += chi[4 * s + k] * chi[4 * s + k];
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < 4) norms[4 * a + threadIdx.x] = dV * red[threadIdx.x][0];
}

// rho[0, n) holds the total guess; on exit rho[0, n) = (1 + z) rho / 2 (up)
// and rho[n, 2n) = (1 - z) rho / 2 (down).
__global__ void k_split_spin_guess(double* rho, long n, double z) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const double r = rho[i];
        rho[i] = 0.5 * (1.0 + z) * r;
        rho[n + i] = 0.5 * (1.0 - z) * r;
    }
}

__global__ void k_scale(double* v, long n, const double* num, double target) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] *= target / *num;
}

// eyez, dy, dz of every sweep pair: the line (slab row, plane) of pair q
// against its candidate's image-shifted centre.  The pair's (slab, plane)
// list is found by binary search in pair_off.
__global__ void k_pair_geometry(SweepPair* pairs, long n, const int* pair_off, int nlists, const CandInfo* cand,
                                int kmax, int nz, int ty, const double* pos, double hy, double hz, double Ly,
                                double Lz, double inv_rc2) {
    long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    int lo = 0, hi = nlists;   // pair_off[lo] <= q < pair_off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (pair_off[mid] <= q) lo = mid;
        else hi = mid;
    }
    const int sl = lo / nz, z = lo - sl * nz;
    SweepPair& P = pairs[q];
    if (P.n == 0) {
        P.eyez = P.dy = P.dz = 0.0;
        return;
    }
    const CandInfo ci = cand[(long)sl * kmax + P.k];
    const double cy = pos[3 * ci.atom + 1] - (double)ci.sy * Ly;
    const double cz = pos[3 * ci.atom + 2] - (double)ci.sz * Lz;
    const double dy = (double)(sl * ty + P.row) * hy - cy;
    const double dz = (double)z * hz - cz;
    P.dy = dy;
    P.dz = dz;
    P.eyez = exp(-(dy * dy + dz * dz) * inv_rc2);
}

__global__ void k_pack_proj_pairs(const SweepPair* pairs, long n, ProjPair* out) {
    long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const SweepPair P = pairs[q];
    ProjPair R;
    R.kw = (uint32_t)P.k | ((uint32_t)P.xo << 10) | ((uint32_t)P.run << 18);
    R.rw = (uint32_t)P.row | ((uint32_t)P.xlo << 8) | ((uint32_t)P.n << 16);
    R.eyez = P.eyez;
    R.dy = P.dy;
    R.dz = P.dz;
    out[q] = R;
}

// ------------------------------------------------------------------ host set-up

static long factorial(int n) {
    long r = 1;
    for (int i = 2; i <= n; ++i) r *= i;
    return r;
}

// Centred second-derivative weights of order 2 n_o:
//   w_q = 2 (-1)^(q+1) (n_o!)^2 / (q^2 (n_o-q)! (n_o+q)!),  w_0 = -2 sum w_q.
static void fd_weights(int n_o, double* w) {
    double s = 0.0;
    for (int q = 1; q <= n_o; ++q) {
        double num = 2.0 * ((q % 2) ? 1.0 : -1.0) * (double)factorial(n_o) * (double)factorial(n_o);
        double den = (double)q * q * (double)factorial(n_o - q) * (double)factorial(n_o + q);
        w[q] = num / den;
        s += w[q];
    }
    w[0] = -2.0 * s;
    for (int q = n_o + 1; q <= kMaxHalfOrder; ++q) w[q] = 0.0;
}

static AtomImages make_images(const sparc_gpu_ctx c, int a, double amp, double width, double rmax) {
    AtomImages A;
    A.x = c->pos[3 * a];
    A.y = c->pos[3 * a + 1];
    A.z = c->pos[3 * a + 2];
    A.amp = amp;
    A.inv_w2 = 1.0 / (width * width);
    A.rmax2 = rmax * rmax;
    double P[3] = {A.x, A.y, A.z}, L[3] = {c->Lx, c->Ly, c->Lz};
    for (int d = 0; d < 3; ++d) {
        // shifts n with |x - P - n L| <= rmax for some x in [0, L)
        A.n0[d] = (int)std::floor((0.0 - P[d] - rmax) / L[d]) - 1;
        A.n1[d] = (int)std::ceil((L[d] - P[d] + rmax) / L[d]) + 1;
    }
    return A;
}

template <typename V>
static sparc_status upload(sparc_gpu_ctx c, V** dst, const std::vector<V>& src) {
    SG_HIP(c, hipMalloc((void**)dst, std::max<size_t>(1, src.size()) * sizeof(V)));
    if (!src.empty())
        SG_HIP(c, hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice, c->stream));
    return SPARC_OK;
}

static sparc_status gaussian_field(sparc_gpu_ctx c, double sign, double* out, bool sad) {
    std::vector<AtomImages> at(c->n_atoms);
    const double pi = 3.14159265358979323846;
    for (int a = 0; a < c->n_atoms; ++a) {
        double w = sad ? c->sad_width : c->rc_loc[a];
        double amp = sign * c->Z[a] * std::pow(pi * w * w, -1.5);
        at[a] = make_images(c, a, amp, w, 8.0 * w);
    }
    AtomImages* d_at = nullptr;
    sparc_status s = upload(c, &d_at, at);
    if (s != SPARC_OK) return s;
    k_gaussian_field<<<div_up(c->nd, 256), 256, 0, c->stream>>>(d_at, c->n_atoms, c->nx, c->ny, c->nz, c->hx, c->hy,
                                                                 c->hz, c->Lx, c->Ly, c->Lz, out);
    SG_CHECK_LAUNCH(c);
    SG_HIP(c, hipStreamSynchronize(c->stream));
    SG_HIP(c, hipFree(d_at));
    return SPARC_OK;
}

// Real orthonormal eigenbasis of the periodic 1D stencil: columns are the
// constant, cos/sin pairs and (N even) the alternating mode.  freq[k] is the
// integer frequency of column k.
static void fourier_basis(int N, std::vector<double>& U, std::vector<int>& freq) {
    const double pi = 3.14159265358979323846;
    U.assign((size_t)N * N, 0.0);
    freq.assign(N, 0);
    int col = 0;
    for (int j = 0; j < N; ++j) U[j + (size_t)N * col] = 1.0 / std::sqrt((double)N);
    freq[col++] = 0;
    for (int k = 1; 2 * k < N; ++k) {
        for (int j = 0; j < N; ++j) {
            double th = 2.0 * pi * (double)k * (double)j / N;
            U[j + (size_t)N * col] = std::sqrt(2.0 / N) * std::cos(th);
            U[j + (size_t)N * (col + 1)] = std::sqrt(2.0 / N) * std::sin(th);
        }
        freq[col] = k;
        freq[col + 1] = k;
        col += 2;
    }
    if (N % 2 == 0) {
        for (int j = 0; j < N; ++j) U[j + (size_t)N * col] = (j % 2 ? -1.0 : 1.0) / std::sqrt((double)N);
        freq[col++] = N / 2;
    }
}

static double symbol(const double* w, int n_o, double th) {
    double s = w[0];
    for (int q = 1; q <= n_o; ++q) s += 2.0 * w[q] * std::cos(q * th);
    return s;
}

// Per-slab tables of the nonlocal sweep.  The grid is cut into y-slabs of
// ty rows.  A candidate of a slab is an (atom, periodic image) pair whose
// support meets the slab; the image shift of a support point is the floor of
// its unwrapped index over the grid size, so every candidate's points lie
// inside the periodic cell.  The support of a candidate on one grid line
// (slab row, plane) is a segment of consecutive x (a ball meets a line in a
// segment); each (plane, candidate, row) segment is a "pair".  Per (slab,
// plane) the pairs are listed by (candidate, row), and point p stores the
// byte indices of its pairs in its plane's list in pe8[p] (0xFF pads).
void free_slab_tables(NonlocalTables& T) {
    for (void* p : {(void*)T.pe8, (void*)T.slab_cand, (void*)T.slab_k, (void*)T.pairs, (void*)T.pair_off,
                    (void*)T.red_off, (void*)T.red_idx, (void*)T.ppairs})
        if (p) hipFree(p);
    T.ppairs = nullptr;
    T.pe8 = nullptr;
    T.slab_cand = nullptr;
    T.slab_k = nullptr;
    T.pairs = nullptr;
    T.pair_off = nullptr;
    T.red_off = nullptr;
    T.red_idx = nullptr;
    T.slab_ty = 0;
}

sparc_status build_pair_tables(sparc_gpu_ctx c, const std::vector<uint32_t>& ent, int ty, NonlocalTables& T) {
    const int nx = c->nx, ny = c->ny, nz = c->nz;
    const int nslab = (ny + ty - 1) / ty;
    // slab-local candidate index of every image entry
    std::vector<std::vector<uint32_t>> cand_key(nslab);
    std::vector<std::vector<CandInfo>> cands(nslab);
    struct Tup {
        uint64_t key;   // (slab, z, k, row) for sorting
        int x;
        long e;         // entry index
    };
    std::vector<Tup> tup;
    tup.reserve(ent.size());
    std::vector<std::unordered_map<uint32_t, int>> kmap(nslab);
    for (long p = 0; p < c->nd; ++p) {
        const int x = (int)(p % nx), y = (int)((p / nx) % ny), z = (int)(p / ((long)nx * ny));
        const int sl = y / ty, row = y - sl * ty;
        for (int e = c->pe_off_host[p]; e < c->pe_off_host[p + 1]; ++e) {
            const uint32_t w = ent[e];
            auto& km = kmap[sl];
            const auto it = km.find(w);
            int k = it == km.end() ? -1 : it->second;
            const int sx = (int)((w >> 20) & 15u) - 8, sz = (int)(w >> 28) - 8;
            const int ix = x + sx * nx, iz = z + sz * nz;
            if (k < 0) {
                k = (int)cands[sl].size();
                km.emplace(w, k);
                CandInfo ci;
                ci.atom = (int)(w & 0xFFFFFu);
                ci.sx = sx;
                ci.sy = (int)((w >> 24) & 15u) - 8;
                ci.sz = sz;
                ci.ixlo = ci.ixhi = ix;
                ci.izlo = ci.izhi = iz;
                cands[sl].push_back(ci);
            }
            CandInfo& ci = cands[sl][k];
            ci.ixlo = std::min(ci.ixlo, ix);
            ci.ixhi = std::max(ci.ixhi, ix);
            ci.izlo = std::min(ci.izlo, iz);
            ci.izhi = std::max(ci.izhi, iz);
            if (k >= 1023 || row >= 63)
                return set_err(c, SPARC_ERR_ARG, "projector overlap too dense for the sweep tables");
            tup.push_back({(((uint64_t)sl * nz + z) << 20) | ((uint64_t)k << 6) | (uint64_t)row, x, e});
        }
    }
    std::sort(tup.begin(), tup.end(), [](const Tup& A, const Tup& B) {
        return A.key < B.key || (A.key == B.key && A.x < B.x);
    });
    // group into pairs; per (slab, plane) the lists are consecutive
    std::vector<SweepPair> pairs;
    std::vector<int> pair_off((size_t)nslab * nz + 1, 0);
    std::vector<int> ent_pair(ent.size(), -1);   // pair index (within its plane list) of every entry
    int pmax = 0;
    size_t i = 0;
    while (i < tup.size()) {
        const uint64_t sz_key = tup[i].key >> 20;
        size_t j = i;
        int npl = 0;
        while (j < tup.size() && (tup[j].key >> 20) == sz_key) {
            size_t q = j;
            while (q < tup.size() && tup[q].key == tup[j].key) ++q;
            const int xlo = tup[j].x, n = (int)(q - j);
            if (tup[q - 1].x != xlo + n - 1)
                return set_err(c, SPARC_ERR_ARG, "projector support is not a segment on a grid line");
            if (n > 255 || xlo > 255) return set_err(c, SPARC_ERR_ARG, "projector segment too long for the sweep tables");
            const int sl = (int)(sz_key / nz);
            SweepPair sp;
            sp.k = (int)((tup[j].key >> 6) & 1023u);
            sp.row = (int)(tup[j].key & 63u);
            sp.xlo = xlo;
            sp.n = n;
            sp.run = 0;
            sp.xo = xlo - (cands[sl][sp.k].ixlo - cands[sl][sp.k].sx * nx);
            sp.eyez = sp.dy = sp.dz = 0.0;
            // run length of the candidate's pairs, held by its first pair; a
            // run never crosses a multiple of 64 in the plane list (empty
            // pairs pad it), so that one wave holds every run it starts
            if (npl == 0 || pairs.back().k != sp.k) {
                int r = 0;
                for (size_t q2 = j; q2 < tup.size() && (tup[q2].key >> 6) == (tup[j].key >> 6); ++q2)
                    if (q2 == j || (tup[q2].key & 63u) != (tup[q2 - 1].key & 63u)) ++r;
                sp.run = r;
                if (npl % 64 + r > 64) {
                    SweepPair pad{};
                    while (npl % 64 != 0) {
                        pairs.push_back(pad);
                        ++npl;
                    }
                }
            }
            if (npl >= 255) return set_err(c, SPARC_ERR_ARG, "more than 255 projector segments in one slab plane");
            if (sp.xo < 0 || sp.xo > 255) return set_err(c, SPARC_ERR_ARG, "projector support wider than 256 points");
            for (size_t r = j; r < q; ++r) ent_pair[tup[r].e] = npl;
            pairs.push_back(sp);
            ++npl;
            j = q;
        }
        pair_off[sz_key + 1] = npl;
        pmax = std::max(pmax, npl);
        i = j;
    }
    for (size_t q = 0; q < (size_t)nslab * nz; ++q) pair_off[q + 1] += pair_off[q];
    // per point: its pairs (at most 7)
    std::vector<uint64_t> pe8(c->nd, ~0ull);
    int max_entries = 0;
    for (long p = 0; p < c->nd; ++p) {
        uint64_t word = ~0ull;
        int cnt = 0;
        for (int e = c->pe_off_host[p]; e < c->pe_off_host[p + 1]; ++e) {
            if (cnt >= 7) return set_err(c, SPARC_ERR_ARG, "more than 7 projector supports meet at one point");
            word &= ~(0xFFull << (8 * cnt));
            word |= (uint64_t)ent_pair[e] << (8 * cnt);
            ++cnt;
        }
        pe8[p] = word;
        max_entries = std::max(max_entries, cnt);
    }
    T.max_entries = max_entries;
    int kmax = 0, xw = 0;
    for (int sl = 0; sl < nslab; ++sl) {
        kmax = std::max(kmax, (int)cands[sl].size());
        for (auto& ci : cands[sl]) xw = std::max(xw, ci.ixhi - ci.ixlo + 1);
    }
    T.slab_kmax = std::max(kmax, 1);
    T.slab_xw = std::max(xw, 1);
    T.pair_max = std::max(pmax, 1);
    std::vector<CandInfo> flat((size_t)nslab * T.slab_kmax);
    std::vector<int> kcount(nslab);
    for (int sl = 0; sl < nslab; ++sl) {
        kcount[sl] = (int)cands[sl].size();
        for (size_t k = 0; k < cands[sl].size(); ++k) flat[(size_t)sl * T.slab_kmax + k] = cands[sl][k];
    }
    // the (slab, candidate) partials of each atom, in (slab, candidate) order
    std::vector<int> red_off(c->n_atoms + 1, 0), red_idx;
    {
        std::vector<std::vector<int>> per_atom(c->n_atoms);
        for (int sl = 0; sl < nslab; ++sl)
            for (size_t k = 0; k < cands[sl].size(); ++k)
                per_atom[cands[sl][k].atom].push_back(sl * T.slab_kmax + (int)k);
        for (int a = 0; a < c->n_atoms; ++a) {
            red_off[a + 1] = red_off[a] + (int)per_atom[a].size();
            red_idx.insert(red_idx.end(), per_atom[a].begin(), per_atom[a].end());
        }
    }
    sparc_status st;
    if ((st = upload(c, &T.pe8, pe8)) != SPARC_OK) return st;
    if ((st = upload(c, &T.slab_cand, flat)) != SPARC_OK) return st;
    if ((st = upload(c, &T.slab_k, kcount)) != SPARC_OK) return st;
    if ((st = upload(c, &T.pairs, pairs)) != SPARC_OK) return st;
    if ((st = upload(c, &T.pair_off, pair_off)) != SPARC_OK) return st;
    if ((st = upload(c, &T.red_off, red_off)) != SPARC_OK) return st;
    if ((st = upload(c, &T.red_idx, red_idx)) != SPARC_OK) return st;
    // geometry of every pair on the device
    if (!pairs.empty()) {
        k_pair_geometry<<<div_up((long)pairs.size(), 256), 256, 0, c->stream>>>(
            T.pairs, (long)pairs.size(), T.pair_off, nslab * nz, T.slab_cand, T.slab_kmax, nz, ty, c->atom_pos,
            c->hy, c->hz, (double)ny * c->hy, (double)nz * c->hz, 1.0 / (c->rc_nl * c->rc_nl));
        SG_CHECK_LAUNCH(c);
        SG_HIP(c, hipMalloc((void**)&T.ppairs, pairs.size() * sizeof(ProjPair)));
        k_pack_proj_pairs<<<div_up((long)pairs.size(), 256), 256, 0, c->stream>>>(T.pairs, (long)pairs.size(),
                                                                                  T.ppairs);
        SG_CHECK_LAUNCH(c);
    }
    T.slab_ty = ty;
    if (c->debug)
        fprintf(stderr, "[sparc_gpu] pair tables: ty %d, %zu pairs, at most %d per plane, %d candidates, ex width %d\n",
                ty, pairs.size(), T.pair_max, T.slab_kmax, T.slab_xw);
    return SPARC_OK;
}

sparc_status build_tables(sparc_gpu_ctx c) {
#pragma clang fp contract(off)
    const double pi = 3.14159265358979323846;
    // --- stencil coefficients of -1/2 Delta_h
    fd_weights(c->n_o, c->w);
    double ix2 = 1.0 / (c->hx * c->hx), iy2 = 1.0 / (c->hy * c->hy), iz2 = 1.0 / (c->hz * c->hz);
    for (int q = 0; q <= kMaxHalfOrder; ++q) {
        c->cf64.cx[q] = -0.5 * c->w[q] * ix2;
        c->cf64.cy[q] = -0.5 * c->w[q] * iy2;
        c->cf64.cz[q] = -0.5 * c->w[q] * iz2;
        c->cf32.cx[q] = (float)c->cf64.cx[q];
        c->cf32.cy[q] = (float)c->cf64.cy[q];
        c->cf32.cz[q] = (float)c->cf64.cz[q];
    }
    c->cf64.c0 = -0.5 * c->w[0] * (ix2 + iy2 + iz2);
    c->cf32.c0 = (float)c->cf64.c0;
    double spi = std::fabs(symbol(c->w, c->n_o, pi));
    c->kin_bound = 0.5 * spi * (ix2 + iy2 + iz2);

    // --- device scalars and flags
    SG_HIP(c, hipMalloc((void**)&c->scal, S_COUNT * sizeof(double)));
    SG_HIP(c, hipMalloc((void**)&c->flags, F_COUNT * sizeof(int)));
    SG_HIP(c, hipMemsetAsync(c->scal, 0, S_COUNT * sizeof(double), c->stream));
    SG_HIP(c, hipMemsetAsync(c->flags, 0, F_COUNT * sizeof(int), c->stream));
    SG_HIP(c, hipMalloc((void**)&c->veff, c->nd * sizeof(double)));
    SG_HIP(c, hipMalloc((void**)&c->veff32, c->nd * sizeof(float)));
    SG_HIP(c, hipMemsetAsync(c->veff, 0, c->nd * sizeof(double), c->stream));
    SG_HIP(c, hipMemsetAsync(c->veff32, 0, c->nd * sizeof(float), c->stream));

    // --- pseudocharge
    SG_HIP(c, hipMalloc((void**)&c->b, c->nd * sizeof(double)));
    sparc_status st = gaussian_field(c, -1.0, c->b, false);
    if (st != SPARC_OK) return st;

    // --- self energy and overlap correction
    {
        std::vector<AtomImages> at(c->n_atoms);
        for (int a = 0; a < c->n_atoms; ++a) {
            double rc = c->rc_loc[a];
            at[a] = make_images(c, a, -c->Z[a] * std::pow(pi * rc * rc, -1.5), rc, 8.0 * rc);
        }
        AtomImages* d_at = nullptr;
        double *d_Z = nullptr, *d_rc = nullptr, *d_pos = nullptr, *d_part = nullptr, *d_sum = nullptr;
        if ((st = upload(c, &d_at, at)) != SPARC_OK) return st;
        if ((st = upload(c, &d_Z, c->Z)) != SPARC_OK) return st;
        if ((st = upload(c, &d_rc, c->rc_loc)) != SPARC_OK) return st;
        if ((st = upload(c, &d_pos, c->pos)) != SPARC_OK) return st;
        long npair = (long)c->n_atoms * c->n_atoms;
        SG_HIP(c, hipMalloc((void**)&d_part, std::max<long>(npair, c->n_atoms) * sizeof(double)));
        SG_HIP(c, hipMalloc((void**)&d_sum, 2 * sizeof(double)));
        k_self_energy<<<c->n_atoms, 256, 0, c->stream>>>(d_at, d_Z, d_rc, c->n_atoms, c->hx, c->hy, c->hz, c->dV,
                                                        d_part);
        SG_CHECK_LAUNCH(c);
        k_sum_serial<<<1, 256, 0, c->stream>>>(d_part, c->n_atoms, d_sum);
        const double rmax = 10.0;
        int nim[3] = {(int)std::ceil(rmax / c->Lx) + 1, (int)std::ceil(rmax / c->Ly) + 1,
                      (int)std::ceil(rmax / c->Lz) + 1};
        k_overlap<<<div_up(npair, 128), 128, 0, c->stream>>>(d_pos, d_Z, d_rc, c->n_atoms, c->Lx, c->Ly, c->Lz, rmax,
                                                            nim[0], nim[1], nim[2], d_part);
        SG_CHECK_LAUNCH(c);
        k_sum_serial<<<1, 256, 0, c->stream>>>(d_part, npair, d_sum + 1);
        double h2[2];
        SG_HIP(c, hipMemcpyAsync(h2, d_sum, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        SG_HIP(c, hipStreamSynchronize(c->stream));
        c->e_self = h2[0];
        c->e_c = h2[1];
        hipFree(d_at);
        hipFree(d_Z);
        hipFree(d_rc);
        hipFree(d_part);
        hipFree(d_sum);
        hipFree(d_pos);
    }

    // --- atom positions for the on-the-fly projector evaluation
    if ((st = upload(c, &c->atom_pos, c->pos)) != SPARC_OK) return st;

    // --- nonlocal projector tables
    if (c->nl_lmax >= 1) {
        sg::NonlocalTables& T = c->nl;
        T.n_atoms = c->n_atoms;
        if (c->n_atoms >= (1 << 20)) return set_err(c, SPARC_ERR_ARG, "too many atoms for the projector tables");
        std::vector<long> sup_off(c->n_atoms + 1, 0);
        std::vector<int> sup_idx, sup_atom, img_off(1, 0), img_ijk;
        std::vector<std::pair<long, uint32_t>> img_pts;  // (flat point, packed atom/image)
        std::vector<long> ip_off(c->n_atoms + 1, 0);
        std::vector<int> ip_idx, box_lo(3 * (size_t)c->n_atoms);
        std::vector<uint32_t> ip_box;
        bool image_overflow = false;
        const double rcut = c->rcut_nl, r2max = rcut * rcut;
        const double h[3] = {c->hx, c->hy, c->hz};
        const int n[3] = {c->nx, c->ny, c->nz};
        for (int a = 0; a < c->n_atoms; ++a) {
            const double* P = &c->pos[3 * a];
            int lo[3], hi[3];
            for (int d = 0; d < 3; ++d) {
                lo[d] = (int)std::ceil((P[d] - rcut) / h[d]);
                hi[d] = (int)std::floor((P[d] + rcut) / h[d]);
            }
            // (flat index, unwrapped i, j, k) of every image point in the ball
            std::vector<std::pair<long, std::array<int, 3>>> pts;
            auto fdiv = [](int v, int m) { return (v >= 0) ? v / m : -((-v + m - 1) / m); };
            for (int k = lo[2]; k <= hi[2]; ++k) {
                double dz = k * h[2] - P[2];
                for (int j = lo[1]; j <= hi[1]; ++j) {
                    double dy = j * h[1] - P[1];
                    for (int i = lo[0]; i <= hi[0]; ++i) {
                        double dx = i * h[0] - P[0];
                        double r2 = dx * dx + dy * dy;
                        r2 = r2 + dz * dz;
                        if (r2 > r2max) continue;
                        int wi = ((i % n[0]) + n[0]) % n[0];
                        int wj = ((j % n[1]) + n[1]) % n[1];
                        int wk = ((k % n[2]) + n[2]) % n[2];
                        long flat = wi + (long)n[0] * (wj + (long)n[1] * wk);
                        pts.push_back({flat, {i, j, k}});
                        // image-level entry of the point: atom and image shifts
                        int sx = fdiv(i, n[0]), sy = fdiv(j, n[1]), sz = fdiv(k, n[2]);
                        if (sx < -8 || sx > 7 || sy < -8 || sy > 7 || sz < -8 || sz > 7) image_overflow = true;
                        img_pts.push_back({flat, (uint32_t)a | ((uint32_t)((sx + 8) & 15) << 20) |
                                                     ((uint32_t)((sy + 8) & 15) << 24) |
                                                     ((uint32_t)((sz + 8) & 15) << 28)});
                    }
                }
            }
            std::stable_sort(pts.begin(), pts.end(),
                             [](const auto& A, const auto& B) { return A.first < B.first; });
            for (int d = 0; d < 3; ++d) {
                box_lo[3 * a + d] = lo[d];
                T.box_ext = std::max(T.box_ext, hi[d] - lo[d] + 1);
            }
            for (auto& q : pts) {
                ip_idx.push_back((int)q.first);
                ip_box.push_back((uint32_t)(q.second[0] - lo[0]) | ((uint32_t)(q.second[1] - lo[1]) << 8) |
                                 ((uint32_t)(q.second[2] - lo[2]) << 16));
            }
            ip_off[a + 1] = (long)ip_idx.size();
            long prev = -1;
            for (auto& q : pts) {
                if (q.first != prev) {
                    if (prev >= 0) img_off.push_back((int)(img_ijk.size() / 3));
                    sup_idx.push_back((int)q.first);
                    sup_atom.push_back(a);
                    prev = q.first;
                }
                img_ijk.push_back(q.second[0]);
                img_ijk.push_back(q.second[1]);
                img_ijk.push_back(q.second[2]);
            }
            if (prev >= 0) img_off.push_back((int)(img_ijk.size() / 3));
            sup_off[a + 1] = (long)sup_idx.size();
            T.max_per_atom = std::max<int>(T.max_per_atom, (int)(sup_off[a + 1] - sup_off[a]));
        }
        T.n_sup = (long)sup_idx.size();
        // image-level point-major entries, atom order within a point
        {
            if (image_overflow)
                return set_err(c, SPARC_ERR_ARG, "projector support spans too many periodic images");
            c->pe_off_host.assign(c->nd + 1, 0);
            for (auto& q : img_pts) c->pe_off_host[q.first + 1]++;
            for (long p = 0; p < c->nd; ++p) c->pe_off_host[p + 1] += c->pe_off_host[p];
            std::vector<uint32_t> ent(img_pts.size());
            std::vector<int> fill(c->pe_off_host.begin(), c->pe_off_host.end() - 1);
            for (auto& q : img_pts) ent[fill[q.first]++] = q.second;
            T.n_pe = (long)ent.size();
            // slab height: from the nonlocal sweep's largest choice down, the
            // first whose tables fit (at most 255 segments per slab plane, the
            // FP64 sweep and the two-wave FP64 projection within 160 KB of LDS)
            for (int ty = choose_sweep_ty(c->nx, c->ny, nl_sweep_max_threads());; --ty) {
                st = build_pair_tables(c, ent, ty, c->nl);
                const NonlocalTables& N = c->nl;
                const size_t lds = st == SPARC_OK
                                       ? std::max(nl_sweep_lds_bytes(ty, c->nx, c->nz, N.slab_kmax, N.slab_xw, 8),
                                                  nl_proj_lds_bytes(ty, c->nx, c->nz, N.slab_kmax, N.slab_xw, 2, 8))
                                       : 0;
                if (st == SPARC_OK && lds <= 160 * 1024) break;
                if (ty <= 1) return st != SPARC_OK ? st : set_err(c, SPARC_ERR_ARG, "projector tables exceed LDS");
                free_slab_tables(c->nl);
                c->err.clear();
            }
            c->nl_ty = c->nl.slab_ty;
            // The FP32 sweep takes slabs of at most 512 threads, like the
            // local FP32 sweep (measured faster than the FP64 slabs: 13.8
            // against 15.8 ms at 120^3, 0.80 against 0.92 ms at 72^3); the
            // projection pass keeps the FP64 tables in both precisions.  If no
            // such slab fits, the FP32 sweep uses the FP64 tables.
            for (int ty = choose_sweep_ty(c->nx, c->ny, 512); ty >= 1 && ty != c->nl_ty; --ty) {
                st = build_pair_tables(c, ent, ty, c->nl32);
                const NonlocalTables& N = c->nl32;
                if (st == SPARC_OK &&
                    nl_sweep_lds_bytes(ty, c->nx, c->nz, N.slab_kmax, N.slab_xw, 4) <= 160 * 1024)
                    break;
                free_slab_tables(c->nl32);
                c->err.clear();
                st = SPARC_OK;
            }
        }
        // Morton order of the atoms (10 bits per axis of the fractional position)
        {
            std::vector<std::pair<uint64_t, int>> key(c->n_atoms);
            const double Ls[3] = {c->Lx, c->Ly, c->Lz};
            for (int a = 0; a < c->n_atoms; ++a) {
                uint64_t k = 0;
                uint32_t q[3];
                for (int d = 0; d < 3; ++d) {
                    double f = c->pos[3 * a + d] / Ls[d];
                    f = f - std::floor(f);
                    q[d] = (uint32_t)std::min(1023.0, std::floor(f * 1024.0));
                }
                for (int bit = 9; bit >= 0; --bit)
                    for (int d = 2; d >= 0; --d) k = (k << 1) | ((q[d] >> bit) & 1u);
                key[a] = {k, a};
            }
            std::sort(key.begin(), key.end());
            std::vector<int> order(c->n_atoms);
            for (int a = 0; a < c->n_atoms; ++a) order[a] = key[a].second;
            if ((st = upload(c, &T.atom_order, order)) != SPARC_OK) return st;
        }
        std::vector<double> g4(4 * c->n_atoms);
        for (int a = 0; a < c->n_atoms; ++a) {
            g4[4 * a] = c->gamma[2 * a];
            g4[4 * a + 1] = g4[4 * a + 2] = g4[4 * a + 3] = c->gamma[2 * a + 1];
        }
        int *d_img_off = nullptr, *d_img_ijk = nullptr, *d_sup_atom = nullptr;
        double* d_pos = nullptr;
        if (T.box_ext > 255) return set_err(c, SPARC_ERR_ARG, "projector support box wider than 255 points");
        if ((st = upload(c, &T.ip_off, ip_off)) != SPARC_OK) return st;
        if ((st = upload(c, &T.ip_idx, ip_idx)) != SPARC_OK) return st;
        if ((st = upload(c, &T.ip_box, ip_box)) != SPARC_OK) return st;
        if ((st = upload(c, &T.box_lo, box_lo)) != SPARC_OK) return st;
        if ((st = upload(c, &T.sup_off, sup_off)) != SPARC_OK) return st;
        if ((st = upload(c, &T.gamma4, g4)) != SPARC_OK) return st;
        if ((st = upload(c, &d_img_off, img_off)) != SPARC_OK) return st;
        if ((st = upload(c, &d_img_ijk, img_ijk)) != SPARC_OK) return st;
        if ((st = upload(c, &d_sup_atom, sup_atom)) != SPARC_OK) return st;
        if ((st = upload(c, &d_pos, c->pos)) != SPARC_OK) return st;
        long ns = std::max<long>(T.n_sup, 1);
        SG_HIP(c, hipMalloc((void**)&T.sup_chi, 4 * ns * sizeof(double)));
        double rc = c->rc_nl;
        double N0 = std::pow(2.0 / (pi * rc * rc), 0.75);
        double N1 = (2.0 / rc) * N0;
        if (T.n_sup > 0) {
            k_projector_values<<<div_up(T.n_sup, 256), 256, 0, c->stream>>>(
                d_img_off, d_img_ijk, d_sup_atom, d_pos, T.n_sup, c->hx, c->hy, c->hz, 1.0 / (rc * rc), N0, N1,
                T.sup_chi);
            SG_CHECK_LAUNCH(c);
        }
        double* d_norms = nullptr;
        SG_HIP(c, hipMalloc((void**)&d_norms, 4 * c->n_atoms * sizeof(double)));
        k_projector_norms<<<c->n_atoms, 256, 0, c->stream>>>(T.sup_off, T.sup_chi, c->dV, d_norms);
        SG_CHECK_LAUNCH(c);
        std::vector<double> norms(4 * c->n_atoms);
        SG_HIP(c, hipMemcpyAsync(norms.data(), d_norms, norms.size() * sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream));
        SG_HIP(c, hipStreamSynchronize(c->stream));
        T.nl_hi = T.nl_lo = 0.0;
        for (int a = 0; a < c->n_atoms; ++a)
            for (int k = 0; k < 4; ++k) {
                T.nl_hi += std::max(g4[4 * a + k], 0.0) * norms[4 * a + k];
                T.nl_lo += std::min(g4[4 * a + k], 0.0) * norms[4 * a + k];
            }
        hipFree(d_norms);
        hipFree(d_img_off);
        hipFree(d_img_ijk);
        hipFree(d_sup_atom);
        hipFree(d_pos);
        SG_HIP(c, hipMalloc((void**)&c->D, std::max<size_t>(1, 4 * (size_t)c->n_atoms * c->n_states) * sizeof(double)));
        SG_HIP(c, hipMalloc((void**)&c->D32, std::max<size_t>(1, 4 * (size_t)c->n_atoms * c->n_states) * sizeof(float)));
    }


    // --- Poisson eigenbases
    {
        std::vector<double> Ux, Uy, Uz;
        std::vector<int> fx, fy, fz;
        fourier_basis(c->nx, Ux, fx);
        fourier_basis(c->ny, Uy, fy);
        fourier_basis(c->nz, Uz, fz);
        std::vector<double> inv(c->nd);
        for (int k = 0; k < c->nz; ++k)
            for (int j = 0; j < c->ny; ++j)
                for (int i = 0; i < c->nx; ++i) {
                    double lam = -symbol(c->w, c->n_o, 2.0 * pi * fx[i] / c->nx) * ix2 -
                                 symbol(c->w, c->n_o, 2.0 * pi * fy[j] / c->ny) * iy2 -
                                 symbol(c->w, c->n_o, 2.0 * pi * fz[k] / c->nz) * iz2;
                    long p = i + (long)c->nx * (j + (long)c->ny * k);
                    inv[p] = (i == 0 && j == 0 && k == 0) ? 0.0 : 4.0 * pi / lam;
                }
        if ((st = upload(c, &c->pois_ux, Ux)) != SPARC_OK) return st;
        if ((st = upload(c, &c->pois_uy, Uy)) != SPARC_OK) return st;
        if ((st = upload(c, &c->pois_uz, Uz)) != SPARC_OK) return st;
        if ((st = upload(c, &c->pois_inv, inv)) != SPARC_OK) return st;
    }
    SG_HIP(c, hipStreamSynchronize(c->stream));
    return SPARC_OK;
}

}  // namespace sg

using namespace sg;

// ------------------------------------------------------------------ ABI

extern "C" {

sparc_status sparc_gpu_create(const sparc_gpu_system* s, void* hip_stream, sparc_gpu_ctx* out) {
    if (!out) return SPARC_ERR_ARG;
    *out = nullptr;
    if (!s) return SPARC_ERR_ARG;
    // The sweep kernels are instantiated for half-width kMaxHalfOrder (lower
    // orders only zero their outer coefficients): their x padding, y halo
    // rows and z ring wrap each index once, which needs 2 kMaxHalfOrder + 1
    // points on every axis whatever the order.
    const int mino = 2 * kMaxHalfOrder + 1;
    if (s->fd_half_order < 1 || s->fd_half_order > kMaxHalfOrder) return SPARC_ERR_ARG;
    for (int d = 0; d < 3; ++d) {
        if (s->n[d] < mino || s->n[d] > 4096) return SPARC_ERR_ARG;
        if (!(s->L[d] > 0.0) || !std::isfinite(s->L[d])) return SPARC_ERR_ARG;
    }
    if (s->n[0] > 256) return SPARC_ERR_ARG;  // an x-row must fit one sweep workgroup
    if ((long)s->n[0] * s->n[1] * s->n[2] > (1L << 31) - 1) return SPARC_ERR_ARG;
    if (s->n_atoms < 0 || (s->n_atoms > 0 && (!s->pos || !s->Z || !s->rc_loc))) return SPARC_ERR_ARG;
    if (s->nl_lmax != -1 && s->nl_lmax != 1) return SPARC_ERR_ARG;
    if (s->nl_lmax == 1 && (!s->gamma || !(s->rc_nl > 0) || !(s->rcut_nl > 0))) return SPARC_ERR_ARG;
    if (s->n_states < 1 || s->n_states > kEighMaxN) return SPARC_ERR_ARG;
    if (!(s->n_electrons > 0.0) || s->n_electrons > 2.0 * s->n_states) return SPARC_ERR_ARG;
    if (!(s->kT > 0.0)) return SPARC_ERR_ARG;
    if (!(s->sad_width > 0.0)) return SPARC_ERR_ARG;
    for (int a = 0; a < s->n_atoms; ++a) {
        if (!(s->rc_loc[a] > 0.0) || !std::isfinite(s->Z[a])) return SPARC_ERR_ARG;
        for (int d = 0; d < 3; ++d)
            if (!std::isfinite(s->pos[3 * a + d])) return SPARC_ERR_ARG;
    }

    sparc_gpu_ctx c = new (std::nothrow) sparc_gpu_ctx_s();
    if (!c) return SPARC_ERR_NOMEM;
    c->nx = s->n[0];
    c->ny = s->n[1];
    c->nz = s->n[2];
    c->nd = (long)c->nx * c->ny * c->nz;
    c->Lx = s->L[0];
    c->Ly = s->L[1];
    c->Lz = s->L[2];
    c->hx = c->Lx / c->nx;
    c->hy = c->Ly / c->ny;
    c->hz = c->Lz / c->nz;
    c->dV = c->hx * c->hy * c->hz;
    c->n_o = s->fd_half_order;
    c->n_atoms = s->n_atoms;
    c->pos.assign(s->pos, s->pos + 3 * s->n_atoms);
    c->Z.assign(s->Z, s->Z + s->n_atoms);
    c->rc_loc.assign(s->rc_loc, s->rc_loc + s->n_atoms);
    c->nl_lmax = s->nl_lmax;
    if (s->nl_lmax == 1) c->gamma.assign(s->gamma, s->gamma + 2 * s->n_atoms);
    c->rc_nl = s->rc_nl;
    c->rcut_nl = s->rcut_nl;
    c->n_states = s->n_states;
    c->n_electrons = s->n_electrons;
    c->kT = s->kT;
    c->rho_floor = s->rho_floor;
    c->sad_width = s->sad_width;
    c->stream = (hipStream_t)hip_stream;
    for (int i = 0; i < 8; ++i) c->ev[i] = nullptr;
    if (const char* e = std::getenv("SPARC_GPU_DEBUG")) c->debug = std::atoi(e);
    if (const char* e = std::getenv("SPARC_GPU_EIG")) c->eig_jacobi = std::string(e) == "jacobi";
    if (const char* e = std::getenv("SPARC_GPU_TRD_MULTI_MIN")) c->trd_multi_min = std::atoi(e);
    if (const char* e = std::getenv("SPARC_GPU_TRD_TAIL")) c->trd_tail = std::max(0, std::atoi(e));
    if (const char* e = std::getenv("SPARC_GPU_CHOL_MULTI_MIN")) c->chol_multi_min = std::atoi(e);
    if (const char* e = std::getenv("SPARC_GPU_STEIN_LDS_MIN_TPW")) c->stein_lds_min_tpw = std::atoi(e);
    if (const char* e = std::getenv("SPARC_GPU_PROJ_NB")) c->proj_nb = std::atoi(e);
    if (const char* e = std::getenv("SPARC_GPU_NL_SLOTS")) c->nl_slots = std::atoi(e);
    if (const char* e = std::getenv("SPARC_GPU_GEMM_TILE")) c->gemm_tile = std::atoi(e);
    if (const char* e = std::getenv("SPARC_GPU_GEMM_NN_COLS")) c->gemm_nn_cols = std::atoi(e);
    if (const char* e = std::getenv("SPARC_GPU_GEMM_NN_ROWS")) c->gemm_nn_rows = std::atoi(e);
    if (const char* e = std::getenv("SPARC_GPU_SWEEP_GROUP")) c->sweep_group = std::atoi(e);
    if (const char* e = std::getenv("SPARC_GPU_CNN_TZ")) {
        const int tz = std::atoi(e);
        if (tz == 0 || tz == 4 || tz == 8) c->cnn_tz = tz;
    }

    int dev = 0;
    sparc_status st = SPARC_OK;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&c->prop, dev);
    for (int i = 0; e == hipSuccess && i < 8; ++i) e = hipEventCreate(&c->ev[i]);
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_scal, S_COUNT * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_flags, F_COUNT * sizeof(int), hipHostMallocDefault);
    if (e != hipSuccess) {
        st = hip_err(c, e, "device query");
    } else {
        st = scratch_init(c, dev);
        if (st == SPARC_OK) st = build_tables(c);
    }
    if (st != SPARC_OK) {
        sparc_gpu_destroy(c);
        return st;
    }
    *out = c;
    return SPARC_OK;
}

sparc_status sparc_gpu_destroy(sparc_gpu_ctx c) {
    if (!c) return SPARC_ERR_ARG;
    hipStreamSynchronize(c->stream);
    void* ptrs[] = {c->veff, c->veff32, c->veff_spin, c->force_tab, c->kp_off, c->kp_ent, c->kp_slot, c->kp_etab,
                    c->kp_tile_off, c->kp_tile_atoms, c->kp_proj, c->chol_dorig,
                    c->kp_bounds, c->kp_wts, c->b, c->pois_ux, c->pois_uy, c->pois_uz, c->pois_inv, c->work, c->D,
                    c->D32, c->gemm_part, c->small, c->red, c->scal, c->flags, c->field, c->nl.sup_off,
                    c->nl.sup_chi, c->nl.gamma4, c->nl.atom_order, c->atom_pos, c->nl.pe8, c->nl.slab_cand,
                    c->nl.slab_k, c->nl.pairs, c->nl.ppairs, c->nl.pair_off, c->nl.red_off, c->nl.red_idx, c->nl_part,
                    c->nl32.pe8, c->nl32.slab_cand, c->nl32.slab_k, c->nl32.pairs, c->nl32.ppairs, c->nl32.pair_off,
                    c->nl32.red_off, c->nl32.red_idx,
                    c->nl.ip_off, c->nl.ip_idx, c->nl.ip_box, c->nl.box_lo};
    for (void* p : ptrs)
        if (p) hipFree(p);
    for (int i = 0; i < 8; ++i)
        if (c->ev[i]) hipEventDestroy(c->ev[i]);
    for (hipEvent_t e : c->prof_pool) hipEventDestroy(e);
    for (hipEvent_t e : c->step_ev) hipEventDestroy(e);
    if (c->h_scal) hipHostFree(c->h_scal);
    if (c->h_flags) hipHostFree(c->h_flags);
    if (c->jac_exec) hipGraphExecDestroy(c->jac_exec);
    if (c->cap_stream) hipStreamDestroy(c->cap_stream);
    delete c;
    return SPARC_OK;
}

const char* sparc_gpu_last_error(sparc_gpu_ctx c) { return c ? c->err.c_str() : "null context"; }

sparc_status sparc_gpu_profile(sparc_gpu_ctx c, int enable) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    if (!enable) {
        sparc_status st = prof_flush(c);
        if (st != SPARC_OK) return st;
    }
    c->prof = enable != 0;
    return SPARC_OK;
}

sparc_status sparc_gpu_profile_read(sparc_gpu_ctx c, int kernel, double* total_ms, long* launches) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    if (kernel < 0 || kernel >= PK_COUNT) return set_err(c, SPARC_ERR_ARG, "profile_read: bad kernel id");
    sparc_status st = prof_flush(c);
    if (st != SPARC_OK) return st;
    if (total_ms) *total_ms = c->prof_ms[kernel];
    if (launches) *launches = c->prof_n[kernel];
    c->prof_ms[kernel] = 0.0;
    c->prof_n[kernel] = 0;
    return SPARC_OK;
}

long sparc_gpu_grid_size(sparc_gpu_ctx c) { return c ? c->nd : 0; }

double sparc_gpu_dV(sparc_gpu_ctx c) { return c ? c->dV : 0.0; }

sparc_status sparc_gpu_set_veff(sparc_gpu_ctx c, const double* d_veff) {
    if (!c) return SPARC_ERR_ARG;
    if (!d_veff) return set_err(c, SPARC_ERR_ARG, "set_veff: null pointer");
    c->err.clear();
    return set_veff_impl(c, d_veff);
}

sparc_status sparc_gpu_pseudocharge(sparc_gpu_ctx c, double* d_b, double* e_self, double* e_c) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    if (d_b) SG_HIP(c, hipMemcpyAsync(d_b, c->b, c->nd * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    if (e_self) *e_self = c->e_self;
    if (e_c) *e_c = c->e_c;
    SG_HIP(c, hipStreamSynchronize(c->stream));
    return SPARC_OK;
}

sparc_status sparc_gpu_sad_density(sparc_gpu_ctx c, double* d_rho) {
    if (!c) return SPARC_ERR_ARG;
    if (!d_rho) return set_err(c, SPARC_ERR_ARG, "sad_density: null pointer");
    c->err.clear();
    sparc_status st = gaussian_field(c, +1.0, d_rho, true);
    if (st != SPARC_OK) return st;
    k_sum_serial<<<1, 256, 0, c->stream>>>(d_rho, c->nd, c->scal + S_RED0);
    SG_CHECK_LAUNCH(c);
    k_scale<<<div_up(c->nd, 256), 256, 0, c->stream>>>(d_rho, c->nd, c->scal + S_RED0, c->n_electrons / c->dV);
    SG_CHECK_LAUNCH(c);
    return SPARC_OK;
}

sparc_status sparc_gpu_sad_density_spin(sparc_gpu_ctx c, double zeta0, double* d_rho2) {
    if (!c) return SPARC_ERR_ARG;
    if (!d_rho2) return set_err(c, SPARC_ERR_ARG, "sad_density_spin: null pointer");
    if (!(zeta0 >= -1.0 && zeta0 <= 1.0)) return set_err(c, SPARC_ERR_ARG, "sad_density_spin: zeta0 outside [-1, 1]");
    sparc_status st = sparc_gpu_sad_density(c, d_rho2);
    if (st != SPARC_OK) return st;
    k_split_spin_guess<<<div_up(c->nd, 256), 256, 0, c->stream>>>(d_rho2, c->nd, zeta0);
    SG_CHECK_LAUNCH(c);
    return SPARC_OK;
}

sparc_status sparc_gpu_spectrum_bounds(sparc_gpu_ctx c, double* lo, double* hi) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    sparc_status st = bounds_impl(c);
    if (st != SPARC_OK) return st;
    double h2[2];
    SG_HIP(c, hipMemcpyAsync(h2, c->scal + S_LO, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    SG_HIP(c, hipStreamSynchronize(c->stream));
    if (lo) *lo = h2[0];
    if (hi) *hi = h2[1];
    return SPARC_OK;
}

}  // extern "C"

