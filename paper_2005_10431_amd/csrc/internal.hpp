// Internal declarations of the MI355X CheFSI library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "sparc_gpu.h"

namespace sg {

constexpr int kMaxHalfOrder = 6;  // stencil half-width instantiated in the kernels

// Finite-difference coefficients of H's kinetic part -1/2 Delta_h along each
// axis: c*[q] multiplies f(p + q e_d) + f(p - q e_d); c0 multiplies f(p).
template <typename T>
struct StencilCoef {
    T cx[kMaxHalfOrder + 1];
    T cy[kMaxHalfOrder + 1];
    T cz[kMaxHalfOrder + 1];
    T c0;
};

// An (atom, periodic image) pair whose projector support meets a slab, with
// the unwrapped x and z index ranges it covers there.
struct CandInfo {
    int atom, sx, sy, sz;
    int ixlo, ixhi, izlo, izhi;
};

// One line segment of a candidate's support in the nonlocal sweep: the
// points x in [xlo, xlo + n) of slab row `row` at one plane z lie in the
// support of slab candidate k; eyez = exp(-(dy^2 + dz^2)/rc^2) with dy, dz the
// line's offsets from the candidate's (image-shifted) centre.  The host
// fills k, row, xlo, n, run, xo; the device the geometry (k_pair_geometry).
// A plane list may hold empty pairs (n = 0), which contribute nothing.
struct SweepPair {
    int k, row, xlo, n;
    int run;   // first pair of a candidate in its plane list: the candidate's pair count; else 0
    int xo;    // index of the segment's first point in the candidate's ex table
    double eyez, dy, dz;
};

// The same pair packed for the projection pass (32 bytes):
// kw = k | xo << 10 | run << 18, rw = row | xlo << 8 | n << 16.
struct ProjPair {
    uint32_t kw, rw;
    double eyez, dy, dz;
};

// Nonlocal projector tables on the device.
//  - projection: the image points of each atom's ball (ip_*), with the
//    projector values evaluated from per-axis Gaussian tables;
//  - apply (inside the sweep): per-slab candidate (atom, image) lists and a
//    per-point word of candidate indices (pe8, slab_*);
//  - spectral bound: projector values per unique support point (sup_*).
struct NonlocalTables {
    int n_atoms = 0;
    long n_sup = 0;
    long* sup_off = nullptr;   // n_atoms + 1: each atom's unique support points
    double* sup_chi = nullptr; // 4 n_sup projector values (summed over images; for the spectral bound)
    double* gamma4 = nullptr;  // 4 n_atoms: (g_s, g_p, g_p, g_p)
    int* atom_order = nullptr; // atoms in space-filling (Morton) order
    // number of image-level (point, atom, image) entries; the sweep's
    // per-slab tables are built from them on the host
    long n_pe = 0;
    // per-slab tables of the nonlocal sweep (see build_pair_tables): the
    // slab's candidate (atom, image) pairs, the line segments (pairs) of each
    // plane sorted by (candidate, row), and per point the byte indices of its
    // pairs in its plane's list (0xFF pads)
    uint64_t* pe8 = nullptr;
    CandInfo* slab_cand = nullptr;          // [n_slabs][slab_kmax]
    int* slab_k = nullptr;                  // candidates per slab
    int slab_kmax = 0, slab_xw = 0;
    SweepPair* pairs = nullptr;             // all segments, plane lists back to back
    ProjPair* ppairs = nullptr;             // the same, packed for the projection pass
    int* pair_off = nullptr;                // n_slabs * nz + 1: list of (slab, plane)
    int pair_max = 0;                       // longest plane list
    // the (slab, candidate) partial projections of one atom, in fixed order:
    // entries slab * slab_kmax + k of red_idx[red_off[a] .. red_off[a + 1])
    int* red_off = nullptr;
    int* red_idx = nullptr;
    int slab_ty = 0;                        // rows per slab of these tables (0: none built)
    int max_entries = 0;                    // most pairs meeting at one point (at most 7)
    double nl_hi = 0.0, nl_lo = 0.0;  // signed spectral bound contributions
    int max_per_atom = 0;
    // image points of each atom's ball for the projection, in grid order:
    // flat index and the packed position in the atom's bounding box
    // (bits 0-7 x, 8-15 y, 16-23 z, relative to box_lo); the projector
    // values are products of per-axis Gaussian tables
    long* ip_off = nullptr;     // n_atoms + 1
    int* ip_idx = nullptr;
    uint32_t* ip_box = nullptr;
    int* box_lo = nullptr;      // 3 n_atoms (unwrapped grid index of the box corner)
    int box_ext = 0;            // largest box edge (points)
};

}  // namespace sg

struct sparc_gpu_ctx_s {
    // geometry
    int nx = 0, ny = 0, nz = 0;
    long nd = 0;
    double hx = 0, hy = 0, hz = 0, dV = 0;
    double Lx = 0, Ly = 0, Lz = 0;
    int n_o = 6;
    double w[sg::kMaxHalfOrder + 1] = {0};
    sg::StencilCoef<double> cf64;
    sg::StencilCoef<float> cf32;
    double kin_bound = 0;    // upper bound of -1/2 Delta_h

    // atoms
    int n_atoms = 0;
    std::vector<double> pos, Z, rc_loc, gamma;
    int nl_lmax = -1;
    double rc_nl = 0, rcut_nl = 0;
    int n_states = 0;
    double n_electrons = 0, kT = 0, rho_floor = 1e-14, sad_width = 1.0;

    hipStream_t stream = nullptr;
    hipDeviceProp_t prop;

    // device fields
    double* veff = nullptr;     // N_d
    float* veff32 = nullptr;    // N_d
    double* veff_spin = nullptr;  // 2 N_d: V_eff of both spins (spin-polarised SCF, allocated on use)
    double* force_tab = nullptr;  // per-atom force table: pos (3n), Z (n), rc (n), gamma (4n); on use
    // Bloch k-points (allocated on use)
    double kvec[3] = {0, 0, 0};   // current k (1/Bohr)
    int sweep_local_only = 0;     // sweeps skip the nonlocal term (Bloch path adds its own)
    int* kp_off = nullptr;        // N_d + 1: point-major projector entries
    uint32_t* kp_ent = nullptr;   // (atom, image) entries
    uint16_t* kp_slot = nullptr;  // per entry: the atom's slot in its point's tile list
    int* kp_tile_off = nullptr;   // per 256-point tile: offsets into kp_tile_atoms
    int* kp_tile_atoms = nullptr; // distinct atoms with entries in each tile
    int kp_tile_max = 0;          // largest tile atom list
    long kp_n_ent = 0;            // number of entries
    double* kp_etab = nullptr;    // per entry: chi_s, chi_px, chi_py, chi_pz, cos, sin at kp_etab_k
    double kp_etab_k[3] = {0, 0, 0};
    int kp_etab_valid = 0;
    double* kp_proj = nullptr;    // n_atoms x ncol x 8 complex projections
    size_t kp_proj_elems = 0;
    double* kp_bounds = nullptr;  // 3 per k-point: filter bounds of the k-point SCF
    int kp_bounds_n = 0;
    double* kp_wts = nullptr;     // per-state k weights of the k-point SCF
    int kp_wts_n = 0;
    std::vector<std::array<double, 5>> kp_bound_cache;  // (k, nonlocal lo, hi)
    double* b = nullptr;        // pseudocharge, N_d
    double e_self = 0, e_c = 0;
    sg::NonlocalTables nl;
    // per-slab tables of the FP32 sweep when its slab height differs (only
    // the per-slab fields are filled; slab_ty 0: it uses nl's)
    sg::NonlocalTables nl32;

    // Poisson: real orthonormal Fourier bases per axis and the operator's
    // eigenvalues on the product basis
    double* pois_ux = nullptr;  // nx*nx
    double* pois_uy = nullptr;
    double* pois_uz = nullptr;
    double* pois_inv = nullptr; // N_d: 4 pi / eigenvalue of -Delta_h (0 for k = 0)

    // workspace (lazily sized)
    void* work = nullptr;       // one block of n_states columns (bytes below)
    size_t work_bytes = 0;
    double* D = nullptr;        // projector coefficients: 4 n_atoms x n_states
    double* nl_part = nullptr;  // projection partials per (z range, slab, candidate)
    double* scratch = nullptr;  // this device's fixed scratch array (allocation-free filter)
    size_t scratch_elems = 0;
    size_t nl_part_elems = 0;
    float* D32 = nullptr;
    double* gemm_part = nullptr; // split-K partials
    size_t gemm_part_elems = 0;
    double* small = nullptr;    // dense subspace matrices
    size_t small_elems = 0;
    double* red = nullptr;      // reduction partials
    size_t red_elems = 0;
    double* scal = nullptr;     // device scalars (filter params, mu, ...)
    int* flags = nullptr;       // device status flags
    double* field = nullptr;    // grid scratch fields (several N_d)
    int n_field = 0;

    hipEvent_t ev[8];
    std::vector<hipEvent_t> step_ev;  // events of one SCF call, read after its single synchronisation
    double* h_scal = nullptr;   // pinned host mirror of scal (S_COUNT), filled by the SCF calls
    int* h_flags = nullptr;     // pinned host mirror of flags (F_COUNT)
    std::string err;

    // captured Jacobi sweep (see dense.hip)
    hipStream_t cap_stream = nullptr;
    int proj_nb = 8;            // SPARC_GPU_PROJ_NB: at most this many orbitals per projection workgroup (2, 4, 8)
    int nl_slots = 0;           // SPARC_GPU_NL_SLOTS=7: FP64 sweep takes 7 nonlocal slots per point (0: by the tables)
    int gemm_tile = 0;          // SPARC_GPU_GEMM_TILE: Gram/projected-H tile edge (128, 160; 0: by size)
    int gemm_nn_cols = 160;     // SPARC_GPU_GEMM_NN_COLS: rotation tile width (160, 288)
    int gemm_nn_rows = 0;       // SPARC_GPU_GEMM_NN_ROWS: rotation tile height (64, 128; 0: 128 FP64, 64 FP32)
    int sweep_group = 4;        // SPARC_GPU_SWEEP_GROUP: orbitals whose copies of a slab the sweep dispatches side by side
    int cnn_tz = 8;             // SPARC_GPU_CNN_TZ: depth of the matrix-core 16 -> 16 convolution tile (4, 8; 0: vector kernel)
    int cnn_per_cu[2][2] = {};  // resident convolution workgroups per CU, by (tile depth 8, MODE)
    hipGraphExec_t jac_exec = nullptr;
    int jac_N = 0;
    double *jac_A = nullptr, *jac_A2 = nullptr, *jac_V = nullptr, *jac_V2 = nullptr;
    int debug = 0;              // SPARC_GPU_DEBUG: diagnostics on stderr
    int eig_jacobi = 0;         // SPARC_GPU_EIG=jacobi: parallel Jacobi instead of tridiagonal
    int trd_multi_min = 320;    // SPARC_GPU_TRD_MULTI_MIN: N from which the reduction uses many workgroups
    int trd_tail = 256;         // SPARC_GPU_TRD_TAIL: trailing size below which one workgroup finishes it
    int stein_lds_min_tpw = 3;  // SPARC_GPU_STEIN_LDS_MIN_TPW: fewest solves per workgroup for the LDS inverse iteration
    int chol_multi_min = 384;   // SPARC_GPU_CHOL_MULTI_MIN: N from which Cholesky updates over many workgroups
    double* chol_dorig = nullptr;  // original diagonal for the many-workgroup Cholesky (kEighMaxN)
    std::vector<int> pe_off_host;  // point offsets of the image-level entries (host)
    int nl_ty = 6;                 // slab height of the nonlocal sweep
    double* atom_pos = nullptr;    // 3 n_atoms

    // kernel timing (sparc_gpu_profile)
    bool prof = false;
    std::vector<hipEvent_t> prof_pool;        // 2 events per recorded launch
    std::vector<int> prof_kernel;             // kernel id per recorded launch
    int prof_used = 0;
    double prof_ms[32] = {0};   // indexed by sg::ProfKernel
    long prof_n[32] = {0};
};

namespace sg {

// ---- error handling -----------------------------------------------------
sparc_status set_err(sparc_gpu_ctx c, sparc_status s, const std::string& msg);
sparc_status hip_err(sparc_gpu_ctx c, hipError_t e, const char* what);

#define SG_HIP(ctx, call)                                             \
    do {                                                              \
        hipError_t _e = (call);                                       \
        if (_e != hipSuccess) return ::sg::hip_err((ctx), _e, #call); \
    } while (0)

#define SG_CHECK_LAUNCH(ctx) SG_HIP(ctx, hipGetLastError())

// ---- workspace ----------------------------------------------------------
sparc_status ensure_work(sparc_gpu_ctx c, size_t bytes);
sparc_status ensure_gemm_part(sparc_gpu_ctx c, size_t elems);
sparc_status ensure_small(sparc_gpu_ctx c, size_t elems);
sparc_status ensure_red(sparc_gpu_ctx c, size_t elems);
sparc_status ensure_fields(sparc_gpu_ctx c, int n);

// Device scalar slots in ctx->scal
enum Scalar {
    S_A = 0, S_B = 1, S_A0 = 2,      // filter bounds
    S_LO = 4, S_HI = 5,              // spectrum bounds of the current H
    S_RED0 = 8,                      // grid reductions (6 slots)
    S_OCC = 16,                      // mu, entropy term, band energy
    S_EIG = 22,                      // eigensolver norms (2 slots)
    S_CNN = 32,                      // warm-start network head sums (6 slots)
    S_PULAY = 40,                    // Pulay weights gamma (SPARC_PULAY_MAX slots)
    S_SPINB = 50,                    // filter bounds a, b, a0 of both spins (6 slots)
    S_COUNT = 64
};
enum Flag {
    F_NOT_SPD = 0, F_EIG_NOCONV = 1, F_FERMI = 2, F_NONFINITE = 3, F_JACOBI_DONE = 4, F_PULAY_SINGULAR = 5,
    F_INPUT_NONFINITE = 6,   // a non-finite value in an SCF call's input density
    F_COUNT = 16
};

// ---- kernels (launchers) -------------------------------------------------
// H application / Chebyshev sweeps. mode: 0 out = H x; 1 first filter step;
// 2 filter step `step` (>= 2) with xprev = X_{k-1} (may alias out).  With
// projectors the sweep applies the projections held in the context's D,
// which launch_projection must have formed from x.
template <typename T>
sparc_status launch_hsweep(sparc_gpu_ctx c, const T* x, T* out, const T* xprev, int ncol, long ldx,
                           int mode, int step);
// D = gamma dV chi^T x, streaming x once over the sweep's slabs.  The
// partial sums go to `part` (part_elems doubles, as many columns at a time
// as fit) when given, else to context memory sized for the whole block.
template <typename T>
sparc_status launch_projection(sparc_gpu_ctx c, const T* x, int ncol, long ldx, double* part = nullptr,
                               size_t part_elems = 0);
// Chebyshev filter of degree m on X (Wk: scratch block); projection partials
// as in launch_projection.
template <typename T>
sparc_status filter_impl(sparc_gpu_ctx c, T* X, T* Wk, int ncol, long ldx, int m, double* part = nullptr,
                         size_t part_elems = 0);
// LDS bytes of a nonlocal sweep workgroup (slab height ty, nz planes, K
// candidates, ex tables xw wide) of element size tsize
size_t nl_sweep_lds_bytes(int ty, int nx, int nz, int K, int xw, size_t tsize);
// LDS bytes of a projection workgroup of NW waves (one orbital each)
size_t nl_proj_lds_bytes(int ty, int nx, int nz, int K, int xw, int NW, size_t tsize);
int nl_sweep_max_threads();   // workgroup size limit of the nonlocal sweep

// C(MxN, col-major, ldc) = alpha * A^T B, A: K x M (lda), B: K x N (ldb),
// T inputs, double output, deterministic split-K.
template <typename T>
sparc_status gemm_tn(sparc_gpu_ctx c, int M, int N, long K, const T* A, long lda, const T* B, long ldb,
                     double alpha, double* C, int ldc, bool symmetric);
// Out(K x N, ldo) = A (K x M, lda) * Bm (M x N, ldb; double, converted to T)
template <typename T>
sparc_status gemm_nn(sparc_gpu_ctx c, long K, int N, int M, const T* A, long lda, const double* Bm, int ldb,
                     T* Out, long ldo);

// Dense subspace algebra (FP64, N x N col-major)
sparc_status dense_cholesky(sparc_gpu_ctx c, double* M, int N, int* flag);
sparc_status dense_tri_inverse_lower(sparc_gpu_ctx c, const double* L, double* Linv, int N);
sparc_status dense_gemm(sparc_gpu_ctx c, char ta, char tb, int N, const double* A, const double* B, double* C);
sparc_status dense_symmetrize(sparc_gpu_ctx c, double* A, int N);
sparc_status dense_eigh(sparc_gpu_ctx c, double* A, int N, double* V, double* eig, double* work);
sparc_status dense_eigh_tridiag(sparc_gpu_ctx c, double* A, int N, double* V, double* eig, double* work);
constexpr int kEighMaxN = 4096;
inline size_t eigh_work_doubles(int N) { return 6 * (size_t)N * N + 320 * (size_t)N + 64; }

// RR core shared by the public entry point and the SCF step; eig on device.
// check: synchronise after the Cholesky factor and return SPARC_ERR_NOT_SPD
// with X unchanged on a non-SPD Gram matrix (the public call); without it the
// flag F_NOT_SPD stays set on the device for the caller's one final read and
// the rest of the step runs on (bounded loops only).
template <typename T>
sparc_status rayleigh_ritz_impl(sparc_gpu_ctx c, T* X, int ncol, long ldx, double* d_eig, bool check);

// Grid-field kernels
sparc_status potential_impl(sparc_gpu_ctx c, const double* rho, double* phi, double* exc, double* vxc,
                            double* veff);
// deg: electrons per state (2 spin-unpolarised, 1 per spin state); wts:
// optional per-state weights (k-point weights), null for 1
sparc_status occupations_impl(sparc_gpu_ctx c, const double* eig, int ncol, double* occ, double* mu,
                              double deg = 2.0, const double* wts = nullptr);
template <typename T>
sparc_status density_impl(sparc_gpu_ctx c, const T* X, int ncol, long ldx, const double* occ, double* rho);
sparc_status set_veff_impl(sparc_gpu_ctx c, const double* d_veff);
sparc_status bounds_impl(sparc_gpu_ctx c);  // writes S_LO / S_HI on device
sparc_status ensure_force_tables(sparc_gpu_ctx c);
// Bloch k-points at c->kvec; blocks hold columns [Re z; Im z] of 2 N_d rows
sparc_status ensure_kp_tables(sparc_gpu_ctx c);
sparc_status kp_nl_bounds(sparc_gpu_ctx c, const double* k, double* nl_lo, double* nl_hi);
sparc_status bloch_bounds_impl(sparc_gpu_ctx c);
template <typename T>
sparc_status bloch_apply_impl(sparc_gpu_ctx c, const T* X, T* Y, int ncol, long ldx);
template <typename T>
sparc_status bloch_filter_impl(sparc_gpu_ctx c, T* X, T* W, int ncol, long ldx, int m);
template <typename T>
sparc_status rayleigh_ritz_k_impl(sparc_gpu_ctx c, T* X, int ncol, long ldx, double* d_eig, bool check);

// Kernel timing: prof_begin returns a slot (or -1 when disabled), prof_end
// records its closing event.
enum ProfKernel {
    PK_SWEEP = 0,    // filter step k >= 2 (reads X_k, X_{k-1}; writes X_{k+1})
    PK_PROJ = 1,     // projections (streaming pass and per-atom sum)
    PK_GEMM_TN = 2,
    PK_GEMM_NN = 3,
    PK_DENSITY = 4,
    PK_SWEEP1 = 5,   // first filter step
    PK_APPLY = 6,    // plain H application
    PK_CHOL = 7,     // Cholesky of the Gram matrix
    PK_TRINV = 8,    // inverse of the Cholesky factor
    PK_EIG = 9,      // subspace eigensolver (all its launches)
    PK_SMALL = 10,   // N_s x N_s products
    PK_COPY = 11,    // block copies
    PK_EIG_TRD = 12, // eigensolver: tridiagonalisation
    PK_EIG_BIS = 13, // eigensolver: eigenvalues of the tridiagonal matrix
    PK_EIG_VEC = 14, // eigensolver: inverse iteration
    PK_EIG_BACK = 15,// eigensolver: back-transformation
    PK_CNN_FWD = 16, // warm-start network forward (all launches)
    PK_CNN_CONV2 = 17,  // its 16 -> 16 convolution
    PK_CNN_BWD = 18, // network gradient (all launches)
    PK_MIX = 19,     // density mixing step (all launches of one step)
    PK_FORCE_LOCAL = 20,  // local and overlap forces
    PK_FORCE_NL = 21,     // nonlocal forces (all orbital blocks)
    PK_BLOCH = 22,        // Bloch H_k application / filter step
    PK_BLOCH_PROJ = 23,   // Bloch projections
    PK_COUNT = 32    // size of the per-context timing tables
};
static_assert(PK_COUNT == sizeof(sparc_gpu_ctx_s::prof_n) / sizeof(long), "timing table size");
int prof_begin(sparc_gpu_ctx c, int kernel, hipStream_t s = nullptr);  // s = null: the context stream
void prof_end(sparc_gpu_ctx c, int slot, hipStream_t s = nullptr);

// Build geometry tables (ctx.hip)
sparc_status build_tables(sparc_gpu_ctx c);
sparc_status build_pair_tables(sparc_gpu_ctx c, const std::vector<uint32_t>& ent, int ty, NonlocalTables& T);
void free_slab_tables(NonlocalTables& T);
// Device address of the fixed scratch array on device `dev` (current),
// looked up once per device and kept in the context.
sparc_status scratch_init(sparc_gpu_ctx c, int dev);
int choose_sweep_ty(int nx, int ny, int max_threads);

inline int div_up(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace sg
