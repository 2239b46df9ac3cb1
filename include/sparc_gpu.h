/*
 * sparc_gpu.h -- C ABI of the MI355X (gfx950) CheFSI library.
 *
 * The library solves the Gamma-point, spin-unpolarised Kohn-Sham problem of
 * Sec. 2 eq. (1) on a uniform periodic real-space grid (Sec. 2.1) with the
 * Chebyshev-filtered subspace iteration (CheFSI) inside each SCF step
 * (Sec. 2.1).  Every entry point below enqueues hand-written HIP kernels on
 * the stream given at creation; nothing is computed on the host except
 * geometry set-up at creation and a handful of scalars.
 *
 * Conventions shared by all entry points
 * --------------------------------------
 *  - Grid: n[0] x n[1] x n[2] points on an orthorhombic cell L[0..2] (Bohr);
 *    point (ix, iy, iz) sits at (ix*hx, iy*hy, iz*hz), h = L/n, and has flat
 *    index p = ix + n[0]*(iy + n[1]*iz).  N_d = n[0]*n[1]*n[2].  Every axis
 *    is periodic and must have at least 13 points (the kernels' stencil
 *    half-width is 6 whatever fd_half_order is); n[0] <= 256.
 *  - Blocks of orbitals ("X") are column-major N_d x ncol arrays with leading
 *    dimension ldx >= N_d: orbital j occupies X[j*ldx .. j*ldx + N_d).  Their
 *    element type is double for SPARC_FP64 and float for SPARC_FP32.
 *  - Inner products carry the trapezoidal weight dV = hx*hy*hz (Sec. 2.1):
 *    an orthonormal block satisfies dV * X^T X = I.
 *  - Pointers named d_* are device addresses owned by the caller (allocated on
 *    the device current at creation); the library never frees them.  Host
 *    pointers are read during the call only.
 *  - Calls are asynchronous on the context's stream unless stated otherwise.
 *    A context is not reentrant: use one context per host thread.
 *  - Arguments are validated on the host before anything is launched; a
 *    rejected call returns SPARC_ERR_ARG and leaves every buffer untouched.
 *    No exceptions cross the ABI and the library never exits the process.
 *    After an error the context remains usable; sparc_gpu_last_error() gives
 *    a message.
 */
#ifndef SPARC_GPU_H
#define SPARC_GPU_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sparc_gpu_ctx_s* sparc_gpu_ctx;

typedef enum {
    SPARC_FP64 = 0, /* orbitals, stencil and subspace GEMMs in double      */
    SPARC_FP32 = 1  /* orbitals, stencil and subspace GEMMs in float; the
                       Cholesky factor, eigensolve, occupations, density
                       accumulation, potential and mixing stay in double   */
} sparc_prec;

typedef enum {
    SPARC_OK = 0,
    SPARC_ERR_ARG = 1,        /* invalid argument (nothing was launched)   */
    SPARC_ERR_HIP = 2,        /* a HIP runtime call failed                 */
    SPARC_ERR_NOMEM = 3,      /* device allocation failed                  */
    SPARC_ERR_NOT_SPD = 4,    /* Gram matrix not numerically positive
                                 definite (rank-deficient block)           */
    SPARC_ERR_EIG = 5,        /* subspace eigensolver did not converge     */
    SPARC_ERR_FERMI = 6,      /* Fermi level bracket failed                */
    SPARC_ERR_NOCONV = 7,     /* iteration limit reached                   */
    SPARC_ERR_NONFINITE = 8,  /* NaN/Inf met in a checked quantity         */
    SPARC_ERR_SINGULAR = 9    /* Pulay normal equations singular           */
} sparc_status;

/*
 * The system: a periodic cell of model atoms.  Each atom I carries a local
 * pseudopotential V_I(r) = -Z_I erf(r/rc_loc_I)/r, represented through its
 * Gaussian pseudocharge in the local real-space electrostatics of Sec. 2.1,
 * and, if nl_lmax = 1, Kleinman-Bylander nonlocal projectors (Sec. 2.1,
 * applied through their outer-product form):
 *   chi_s  = N0 exp(-r^2/rc_nl^2),  chi_p{x,y,z} = N1 {x,y,z} exp(-r^2/rc_nl^2),
 *   N0 = (2/(pi rc_nl^2))^(3/4),  N1 = (2/rc_nl) N0,  cut at r <= rcut_nl,
 *   summed over periodic images, with energies gamma[I*2 + 0] (s) and
 *   gamma[I*2 + 1] (p, shared by x, y, z).
 * The struct and its arrays are copied by sparc_gpu_create().
 */
typedef struct {
    int n[3];               /* grid points per axis                          */
    double L[3];            /* cell lengths (Bohr)                           */
    int fd_half_order;      /* n_o: 2*n_o-th order centred differences, 1..6  */
    int n_atoms;
    const double* pos;      /* [3*n_atoms] positions (Bohr)                  */
    const double* Z;        /* [n_atoms] valence charges                     */
    const double* rc_loc;   /* [n_atoms] local Gaussian widths (Bohr)        */
    int nl_lmax;            /* -1: no nonlocal part; 1: s and p projectors   */
    const double* gamma;    /* [2*n_atoms] projector energies (Ha); NULL if nl_lmax = -1 */
    double rc_nl;           /* projector Gaussian width (Bohr)               */
    double rcut_nl;         /* projector support radius (Bohr)               */
    int n_states;           /* N_s: columns of the orbital block, <= 4096    */
    double n_electrons;     /* N_e, 0 < N_e < 2*N_s                          */
    double kT;              /* Fermi-Dirac smearing (Ha), > 0                */
    double rho_floor;       /* density floor inside the LDA (e.g. 1e-14)     */
    double sad_width;       /* width (Bohr) of the atomic model densities     */
} sparc_gpu_system;

/* Create a context on the current device: copies the system, builds the
 * finite-difference coefficients, the pseudocharge b, the projector tables
 * and the self/overlap energies.  hip_stream may be NULL (default stream).
 * Synchronous.  Errors: SPARC_ERR_ARG (bad system), SPARC_ERR_NOMEM,
 * SPARC_ERR_HIP. */
sparc_status sparc_gpu_create(const sparc_gpu_system* sys, void* hip_stream, sparc_gpu_ctx* out);

/* Free every device resource of the context (synchronises its stream). */
sparc_status sparc_gpu_destroy(sparc_gpu_ctx ctx);

/* Message describing the last error on this context ("" if none).  The
 * string is owned by the context and valid until its next call. */
const char* sparc_gpu_last_error(sparc_gpu_ctx ctx);

/* Number of grid points N_d and the trapezoidal weight dV. */
long sparc_gpu_grid_size(sparc_gpu_ctx ctx);
double sparc_gpu_dV(sparc_gpu_ctx ctx);

/* Set the effective potential V_eff (Sec. 2 eq. (1)) used by every H
 * application: d_veff is N_d doubles, copied into the context. */
sparc_status sparc_gpu_set_veff(sparc_gpu_ctx ctx, const double* d_veff);

/* Y = H X  (Sec. 2 eq. (1), matrix-free per Sec. 2.1):
 *   H x = -1/2 Delta_h x + V_eff x + sum_I sum_lm gamma_Il chi_Ilm (dV chi_Ilm^T x).
 * d_X, d_Y: N_d x ncol blocks (ldx) of the given precision; they must not
 * overlap.  1 <= ncol <= n_states. */
sparc_status sparc_gpu_apply_H(sparc_gpu_ctx ctx, sparc_prec prec, const void* d_X, void* d_Y,
                               int ncol, long ldx);

/* Scaled Chebyshev filter of degree m >= 1 (the CheFSI filter named in
 * Sec. 2.1): overwrites X with p_m(H) X where, on an eigenvector of H with
 * eigenvalue lam, p_m(lam) = T_m((lam - c)/e) / T_m((a0 - c)/e),
 * e = (b - a)/2, c = (b + a)/2.  Requires a0 < a < b.  d_work is caller
 * scratch of the same shape and precision as X (contents destroyed). */
sparc_status sparc_gpu_chebyshev_filter(sparc_gpu_ctx ctx, sparc_prec prec, void* d_X, void* d_work,
                                        int ncol, long ldx, int degree, double a, double b, double a0);

/* The Chebyshev filter above for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc): same arguments, results and errors as
 * sparc_gpu_chebyshev_filter, bitwise equal to it, and it calls no hipMalloc,
 * hipFree or other allocating routine (nor records timing events).  Its
 * projection partials live in a fixed 32 MiB device array of the library
 * (one copy per GPU, held until the process ends, its address looked up at
 * sparc_gpu_create); columns are processed in as many groups as that needs.
 * Returns SPARC_ERR_ARG when the partials of one column alone exceed the
 * array (4 x (z ranges) x (y-slabs) x (candidates per slab) doubles).  Every
 * entry it reads is written by the same call first, so nothing needs
 * clearing; calls that overlap on one GPU (other streams, other contexts)
 * share the array and race. */
sparc_status sparc_gpu_chebyshev_filter_noalloc(sparc_gpu_ctx ctx, sparc_prec prec, void* d_X, void* d_work,
                                                int ncol, long ldx, int degree, double a, double b, double a0);

/* Orthonormalise and Rayleigh-Ritz (the subspace step of CheFSI, Sec. 2.1):
 *   M = dV Y^T Y = R^T R (Cholesky, FP64), Hs = R^-T (dV Y^T H Y) R^-1,
 *   Hs = Q diag(lam) Q^T (FP64 eigensolver, ascending), X <- Y R^-1 Q.
 * Gram and projected-Hamiltonian products and the rotation run in the block's
 * precision (FP32 MFMA with FP32 accumulation inside K-tiles, FP64 across
 * them, for SPARC_FP32).  d_eig receives ncol doubles.  Synchronises the
 * stream once to report SPARC_ERR_NOT_SPD / SPARC_ERR_EIG; on such an error X
 * is left unchanged.  Uses context-owned workspace (one block). */
sparc_status sparc_gpu_rayleigh_ritz(sparc_gpu_ctx ctx, sparc_prec prec, void* d_X, int ncol, long ldx,
                                     double* d_eig);

/* Dense symmetric eigensolver used inside Rayleigh-Ritz (FP64): on the n x n
 * column-major matrix d_A (destroyed; only the lower triangle is read)
 * returns ascending eigenvalues d_eig (n) and orthonormal eigenvectors as
 * the columns of d_V (n x n).  Householder tridiagonalisation, bisection and
 * inverse iteration (or parallel Jacobi when SPARC_GPU_EIG=jacobi is set at
 * context creation).  1 <= n <= 4096.  Synchronises the stream. */
sparc_status sparc_gpu_subspace_eigh(sparc_gpu_ctx ctx, double* d_A, int n, double* d_V, double* d_eig);

/* Electron density, Sec. 2 eq. (2): rho(p) = sum_j occ[j] X(p, j)^2,
 * accumulated in FP64.  d_occ: ncol doubles; d_rho: N_d doubles. */
sparc_status sparc_gpu_density(sparc_gpu_ctx ctx, sparc_prec prec, const void* d_X, int ncol, long ldx,
                               const double* d_occ, double* d_rho);

/* Fermi-Dirac occupations (Sec. 2: g_j = 2 f_j for the unpolarised case):
 * bisection for mu on [lam_min - 40 kT, lam_max + 40 kT] until
 * |sum g - N_e| < 1e-13.  d_eig, d_occ: ncol doubles; d_mu: 1 double (may
 * be NULL).  Requires 0 < N_e <= 2 ncol. */
sparc_status sparc_gpu_occupations(sparc_gpu_ctx ctx, const double* d_eig, int ncol, double* d_occ,
                                   double* d_mu);

/* Electrostatic and exchange-correlation potentials for density d_rho
 * (Sec. 2.1): phi solves -Delta_h phi = 4 pi (rho + b - mean(rho + b)) with
 * mean(phi) = 0 on the periodic grid; LDA (Slater exchange, PW92
 * correlation).  Outputs (each N_d doubles, any may be NULL): phi, eps_xc,
 * v_xc, V_eff = phi + v_xc.  Does not change the context's V_eff. */
sparc_status sparc_gpu_potential(sparc_gpu_ctx ctx, const double* d_rho, double* d_phi, double* d_exc,
                                 double* d_vxc, double* d_veff);

/* Geometry-derived fields and constants: pseudocharge b (N_d doubles, may
 * be NULL), Gaussian self energy E_self and the point-ion overlap correction
 * E_c (host doubles, may be NULL).  Synchronous. */
sparc_status sparc_gpu_pseudocharge(sparc_gpu_ctx ctx, double* d_b, double* e_self, double* e_c);

/* Superposition-of-atomic-densities guess (Sec. 2.1): a normalised Gaussian of
 * width sad_width carrying Z_I electrons per atom, rescaled so that
 * dV sum rho = N_e.  d_rho: N_d doubles. */
sparc_status sparc_gpu_sad_density(sparc_gpu_ctx ctx, double* d_rho);

/* The same guess split over two spins (eq. (1)-(2) carry a spin index; the
 * spin-polarised SCF mixes both components, Sec. 2.1) by a starting
 * polarisation zeta0 in [-1, 1]: d_rho2[0, N_d) = (1 + zeta0) rho / 2 (up),
 * d_rho2[N_d, 2 N_d) = (1 - zeta0) rho / 2 (down), with rho the output of
 * sparc_gpu_sad_density.  d_rho2: 2 N_d doubles.  Errors: SPARC_ERR_ARG (null
 * pointer, zeta0 outside [-1, 1] or not finite). */
sparc_status sparc_gpu_sad_density_spin(sparc_gpu_ctx ctx, double zeta0, double* d_rho2);

/* Bounds lo <= spec(H) <= hi of the current H (kinetic symbol bound,
 * V_eff extrema, signed projector norms).  Synchronous. */
sparc_status sparc_gpu_spectrum_bounds(sparc_gpu_ctx ctx, double* lo, double* hi);

/* Density mixing (Sec. 2.1: the restarted form of periodic Pulay mixing
 * with a real-space preconditioner) for SCF iteration `iter` (0-based), with
 * x = d_rho_in (updated in place) and f = d_rho_out - d_rho_in, vectors of
 * n_spin x N_d doubles (n_spin = 2: the up then the down spin density; the
 * paper mixes both spin components as one vector of twice the length):
 *   linear step:  x <- x + beta P f
 *   Pulay step, taken when m > 0, the history holds c >= 1 pairs and
 *   (iter + 1) is a multiple of `period`:
 *     gamma = argmin_g || f - dF g ||_2 (normal equations dF^T dF gamma =
 *             dF^T f, solved by LU with partial pivoting),
 *     x <- x - dX gamma + beta P (f - dF gamma),
 *   where dX, dF hold the last c differences x_j - x_{j-1}, f_j - f_{j-1}
 *   (c <= m; each call with iter >= 1 adds the pair for that iteration).
 *   restart = 1: after a Pulay step that used c = m pairs the history is
 *   emptied (the paper names the restarted form without stating the rule;
 *   this is the reading implemented).
 * P = (-Lap_h)(-Lap_h + q0^2)^-1 in the eigenbasis of the discrete Laplacian
 * (constant mode removed) when kerker_q0 > 0, else the identity.  With
 * n_spin = 2, P acts on the total f_up + f_dn and passes the magnetisation
 * part f_up - f_dn unchanged.
 * d_hist (m > 0): (2 m + 2) x n_spin N_d doubles, caller-owned, layout
 * [x_prev | f_prev | dX slots 0..m-1 | dF slots 0..m-1]; the call with
 * iter = 0 initialises it and every call with iter = k must follow the call
 * with k - 1 on the same buffer.  NULL allowed when m = 0.
 * Errors: SPARC_ERR_ARG (m outside [0, SPARC_PULAY_MAX], period < 1, bad
 * beta or q0, n_spin not 1 or 2, null buffers, iter < 0); SPARC_ERR_SINGULAR
 * when a pivot of
 * the normal equations is zero or gamma is not finite (x then holds the
 * linear step, gamma = 0).  Synchronises once. */
#define SPARC_PULAY_MAX 10
sparc_status sparc_gpu_mix(sparc_gpu_ctx ctx, double* d_rho_in, const double* d_rho_out, int n_spin, double beta,
                           double kerker_q0, int pulay_history, int pulay_period, int restart, double* d_hist,
                           int iter);

/* State carried across SCF iterations; every device buffer is caller-owned. */
typedef struct {
    double* d_rho_in;   /* in: rho_in of this iteration; out: mixed density   */
    void* d_X;          /* in/out: N_d x n_states block (ldx, prec)          */
    long ldx;
    int prec;           /* sparc_prec of d_X                                 */
    int cheb_degree;    /* m                                                  */
    int n_first;        /* filter + RR passes in the first iteration (>= 1)  */
    double mix_beta;    /* linear mixing factor, 0 < beta <= 1                */
    double kerker_q0;   /* >= 0: mixing preconditioner wavenumber (1/Bohr);
                           0 = plain linear mixing.  With q0 > 0 the residual
                           is filtered by (-Lap_h)(-Lap_h + q0^2)^-1 before
                           it is mixed (a Kerker-type preconditioner, in the
                           spirit of the real-space preconditioner of
                           Sec. 2.1).                                          */
    int pulay_history;  /* m in [0, SPARC_PULAY_MAX]; 0 = linear mixing only.
                           m > 0: periodic Pulay mixing (sparc_gpu_mix).     */
    int pulay_period;   /* >= 1 (used when m > 0)                            */
    int pulay_restart;  /* 0 or 1: restarted form (used when m > 0)          */
    double* d_pulay;    /* m > 0: (2 m + 2) N_d doubles of mixing history,
                           caller-owned, carried from call to call; may be
                           NULL when m = 0                                   */
    int iter;           /* 0 on the first call; incremented by each call     */
    double* d_eig;      /* out: n_states Ritz values (ascending)             */
    double* d_occ;      /* out: n_states occupations                          */
    double* d_rho_out;  /* optional out: N_d output density (may be NULL)    */
    double bounds[3];   /* a, b, a0 of the last filter (in/out)              */
} sparc_gpu_scf_state;

/* What one SCF iteration reports (energies in Ha, times in ms of device
 * time measured with HIP events on the context's stream). */
typedef struct {
    double free_energy;   /* Harris-Foulkes free energy at rho_in            */
    double band, exc, vxc_dc, elec, self_energy, overlap, entropy; /* terms  */
    double mu;            /* Fermi level                                     */
    double residual;      /* ||rho_out - rho_in|| / ||rho_out||              */
    double t_potential_ms, t_filter_ms, t_rr_ms, t_density_ms, t_total_ms;
    int n_passes;         /* filter + RR passes performed                    */
    int iter;             /* index of this iteration                         */
} sparc_gpu_scf_report;

/* One SCF iteration (Sec. 2.1): V_eff from rho_in (Poisson + LDA); on the
 * first iteration a Rayleigh-Ritz of the starting block, then n_first passes
 * (later iterations: one pass) of Chebyshev filter + Rayleigh-Ritz with
 * a = largest and a0 = smallest Ritz value of the preceding step (a0 = lower
 * spectrum bound before the first filter) and b = upper spectrum bound;
 * occupations, rho_out (Sec. 2 eq. (2)), the free energy at rho_in, the
 * residual, and the mixing step of sparc_gpu_mix with st's mixing fields
 * (plain linear mixing rho_in <- rho_in + beta (rho_out - rho_in) when
 * pulay_history = 0 and kerker_q0 = 0).
 * Synchronises once, at the end, to read the device status flags and fill
 * rep (may be NULL): nothing in the step waits on the host before that.
 * Errors found on the device are reported then, in this order:
 * SPARC_ERR_NONFINITE (NaN or Inf in rho_in), SPARC_ERR_NOT_SPD (a Gram
 * matrix of the block was not positive definite), SPARC_ERR_FERMI,
 * SPARC_ERR_SINGULAR, SPARC_ERR_NONFINITE (non-finite energy or residual).
 * After such an error the step has run to its end on the bad values: X,
 * rho_in, eig and occ hold unspecified values, st->iter and st->bounds are
 * not advanced, and the context stays usable for a fresh state. */
sparc_status sparc_gpu_scf_step(sparc_gpu_ctx ctx, sparc_gpu_scf_state* st, sparc_gpu_scf_report* rep);

/* After an SCF run in SPARC_FP32: promote st->d_X into the FP64 block d_X64
 * (N_d x n_states, leading dimension ldx64), perform one FP64 Rayleigh-Ritz
 * with V_eff from st->d_rho_in, then occupations, rho_out and the free
 * energy at rho_in.  No mixing; st->iter unchanged.  Synchronises once. */
sparc_status sparc_gpu_final_rr_fp64(sparc_gpu_ctx ctx, sparc_gpu_scf_state* st, double* d_X64, long ldx64,
                                     sparc_gpu_scf_report* rep);

/* ---- Spin-polarised form (eq. (1)-(2) with a spin index; Sec. 2.1) -------
 * One orbital block per spin, each with n_states columns; the Hamiltonian
 * of spin s has V_eff^s = phi + v_xc^s(rho_up, rho_dn) with phi from the
 * total density; occupations are one electron per state with a common
 * Fermi level; rho^s = sum_n f_n^s |psi_n^s|^2.  LSDA: exchange by the exact
 * spin-scaling relation, correlation by the PW92 interpolation in
 * zeta = (rho_up - rho_dn) / rho; each spin density is floored at
 * rho_floor / 2. */

/* phi (N_d), eps_xc (N_d), v_xc (2 N_d: up, down) and V_eff (2 N_d) for the
 * spin densities d_rho (2 N_d: up, down).  Outputs may be NULL.  Uses the
 * context's scratch fields. */
sparc_status sparc_gpu_potential_spin(sparc_gpu_ctx ctx, const double* d_rho, double* d_phi, double* d_exc,
                                      double* d_vxc, double* d_veff);

/* Occupations of 2 x ncol spin states: d_eig holds the ncol up then the ncol
 * down eigenvalues; d_occ receives f in the same order (one electron per
 * state), mu by bisection with sum f = N_e; *d_mu (device, may be NULL).
 * Errors: SPARC_ERR_ARG (ncol outside [1, n_states], N_e > 2 ncol). */
sparc_status sparc_gpu_occupations_spin(sparc_gpu_ctx ctx, const double* d_eig, int ncol, double* d_occ,
                                        double* d_mu);

typedef struct {
    double* d_rho_in;   /* in/out: 2 N_d doubles, rho_up then rho_dn         */
    void* d_X_up;       /* in/out: N_d x n_states block of the up spin       */
    void* d_X_dn;       /* in/out: same for the down spin (no overlap)       */
    long ldx;           /* leading dimension of both blocks                  */
    int prec;           /* sparc_prec of both blocks                         */
    int cheb_degree;
    int n_first;
    double mix_beta;
    double kerker_q0;   /* on the total density of the mixing vector         */
    int pulay_history;  /* as in sparc_gpu_scf_state, over 2 N_d vectors     */
    int pulay_period;
    int pulay_restart;
    double* d_pulay;    /* m > 0: (2 m + 2) x 2 N_d doubles, caller-owned    */
    int iter;
    double* d_eig;      /* out: 2 n_states Ritz values (up, then down)       */
    double* d_occ;      /* out: 2 n_states occupations                       */
    double* d_rho_out;  /* optional out: 2 N_d (may be NULL)                 */
    double bounds[6];   /* a, b, a0 of the up spin, then of the down spin    */
} sparc_gpu_scf_spin_state;

/* One spin-polarised SCF iteration: V_eff^up, V_eff^dn from rho_in; for
 * each spin the filter + Rayleigh-Ritz schedule of sparc_gpu_scf_step with
 * that spin's V_eff, block and bounds; common-mu occupations, both output
 * densities, the free energy at rho_in (band and entropy terms over all
 * spin states, v_xc double counting per spin), the residual over the
 * 2 N_d vector and the mixing step of sparc_gpu_mix with n_spin = 2.
 * The context's V_eff holds the down spin's potential afterwards.
 * Synchronises once at the end to fill rep (may be NULL). */
sparc_status sparc_gpu_scf_step_spin(sparc_gpu_ctx ctx, sparc_gpu_scf_spin_state* st, sparc_gpu_scf_report* rep);

/* ---- Bloch k-points (Sec. 2.1) ----------------------------------------------
 * Orbitals obey psi(x + nL) = exp(i k . nL) psi(x); for one k
 *   H_k z = -1/2 Lap_h^k z + V_eff z + sum_I sum_lm gamma_Il chi~_Ilm <chi~_Ilm, z>
 * with the stencil's neighbours past a face taken from the image times
 * exp(+-i k_d L_d), chi~_Ilm(x) = sum_s chi_lm(x + sL - R_I) exp(-i k . sL) over
 * the periodic images s, and <a, b> = dV sum conj(a) b.
 * Layout: a complex orbital z = u + i v is one real column [u ; v] of 2 N_d
 * values (leading dimension ldx >= 2 N_d).  On such columns H_k is the real
 * symmetric operator [[Re H_k, -Im H_k], [Im H_k, Re H_k]]; the k-point
 * filter and Rayleigh-Ritz are the Gamma ones on 2 N_d rows, so a block
 * whose span is closed under z -> i z (columns in pairs [u; v], [-v; u])
 * yields every Bloch eigenvalue twice.  Up to 2 n_states columns per block.
 * k: host array of 3 doubles (1/Bohr).  The last k used stays set in the
 * context (the V_eff of sparc_gpu_set_veff / the SCF applies). */
sparc_status sparc_gpu_apply_H_k(sparc_gpu_ctx ctx, const double* k, sparc_prec prec, const void* d_X, void* d_Y,
                                 int ncol, long ldx);
sparc_status sparc_gpu_chebyshev_filter_k(sparc_gpu_ctx ctx, const double* k, sparc_prec prec, void* d_X,
                                          void* d_work, int ncol, long ldx, int degree, double a, double b,
                                          double a0);
/* Ascending Ritz values of the block (each Bloch eigenvalue of a
 * z -> i z closed span appears twice); X is rotated to the Ritz vectors. */
sparc_status sparc_gpu_rayleigh_ritz_k(sparc_gpu_ctx ctx, const double* k, sparc_prec prec, void* d_X, int ncol,
                                       long ldx, double* d_eig);
/* lo <= spec(H_k) <= hi: V_eff extrema, kinetic symbol bound and the signed
 * k-dependent projector norms dV ||chi~||^2.  Synchronous. */
sparc_status sparc_gpu_spectrum_bounds_k(sparc_gpu_ctx ctx, const double* k, double* lo, double* hi);

typedef struct {
    int n_k;                /* number of k-points (1 .. 4096)                  */
    const double* kpts;     /* host: 3 n_k (1/Bohr)                            */
    const double* kweights; /* host: n_k positive weights summing to 1         */
    void* const* d_X;       /* host array of n_k device blocks, 2 n_states
                               Bloch columns each (ldx, prec)                  */
    long ldx;               /* >= 2 N_d                                        */
    int prec;
    int cheb_degree;
    int n_first;
    double mix_beta;
    double kerker_q0;
    int pulay_history;
    int pulay_period;
    int pulay_restart;
    double* d_pulay;        /* m > 0: (2 m + 2) N_d doubles                    */
    double* d_rho_in;       /* in/out: N_d                                     */
    int iter;
    double* d_eig;          /* out: n_k x 2 n_states Ritz values               */
    double* d_occ;          /* out: n_k x 2 n_states occupations f per column  */
    double* d_rho_out;      /* optional out: N_d                               */
    double* bounds;         /* host in/out: (a, b, a0) per k-point             */
} sparc_gpu_scf_k_state;

/* One SCF iteration over a k-point set: V_eff from rho_in; per k the filter
 * + Rayleigh-Ritz schedule of sparc_gpu_scf_step with H_k and that k's
 * bounds; one Fermi level with sum_k w_k sum_j f_jk = N_e over the Bloch
 * columns (the 2 f_n of a spin-unpolarised state is split over its two
 * columns [u; v], [-v; u]); rho_out
 * = sum_k w_k sum_j f_jk (u_j^2 + v_j^2); the free energy at rho_in with the
 * k-weighted band and entropy terms; the residual and the mixing step of
 * sparc_gpu_mix.  Synchronises once at the end. */
sparc_status sparc_gpu_scf_step_k(sparc_gpu_ctx ctx, sparc_gpu_scf_k_state* st, sparc_gpu_scf_report* rep);

/* ---- Atomic forces ---------------------------------------------------------
 * Hellmann-Feynman forces (Sec. 2: the forces that drive structural
 * relaxation and molecular dynamics): at self-consistency the negative
 * gradient of the free energy with respect to the atom positions has only
 * explicit contributions,
 *   local:    dV sum_x phi(x) grad b_I(x - R_I) - 1/2 dV sum grad(b_I V_I)
 *             (pseudocharge in the electrostatic potential, and the grid
 *             quadrature of the self energy over the atom's 8 rc ball),
 *   overlap:  sum_{J,n}' Z_I Z_J u'(d) (R_J + nL - R_I)/d, u(d) = erfc(d/s)/d,
 *             s = sqrt(rc_I^2 + rc_J^2), images with d < 10 Bohr,
 *   nonlocal: 2 sum_n w_n sum_k gamma_Ik (dV chi_Ik^T psi_n)(dV (grad chi_Ik)^T psi_n)
 *             over the projectors' (point, image) pairs within rcut_nl.
 * d_phi: N_d electrostatic potential of the self-consistent density (from
 * sparc_gpu_potential or sparc_gpu_potential_spin).  d_X: host array of
 * n_blocks device pointers to N_d x ncol orbital blocks (ldx, prec): one
 * block spin-unpolarised, or the up and down blocks (n_blocks = 0 skips the
 * nonlocal part).  d_occ: n_blocks x ncol weights w_n (g_n = 2 f_n
 * unpolarised, f_n per spin block).  d_forces: 3 n_atoms doubles (atom-major
 * x, y, z), Ha/Bohr, overwritten.  Uses the context's scratch reductions;
 * stream-ordered, no synchronisation.
 * Errors: SPARC_ERR_ARG (null pointers, n_blocks outside 0..2, ncol outside
 * [1, n_states], ldx < N_d, bad precision). */
sparc_status sparc_gpu_forces(sparc_gpu_ctx ctx, const double* d_phi, sparc_prec prec, const void* const* d_X,
                              int n_blocks, int ncol, long ldx, const double* d_occ, double* d_forces);

/* Kernel timing (tracing aid).  When enabled, every launch of the listed
 * kernels is bracketed by HIP events on the context's stream.
 * sparc_gpu_profile_read() synchronises, returns the summed device time (ms)
 * and launch count since the last read for one kernel, and resets it.
 * Kernel ids: 0 filter sweep of degree >= 2, 1 nonlocal projection (its
 * streaming pass and per-atom sum),
 * 2 Gram/projected-H GEMM, 3 rotation GEMM, 4 density, 5 first filter
 * sweep, 6 plain H application, 7 Cholesky, 8 triangular inverse,
 * 9 subspace eigensolver (all its launches, host waits included),
 * 10 small N_s x N_s products, 11 block copy-back, 12 tridiagonalisation,
 * 13 tridiagonal eigenvalues, 14 inverse iteration, 15 back-transformation
 * (12-15 are the phases inside 9), 16 warm-start network forward,
 * 17 its 16 -> 16 convolution, 18 network gradient, 19 density mixing
 * step of the SCF (linear with preconditioner, or Pulay; the plain linear
 * step is fused into the energy pass and not listed), 20 local and overlap
 * forces, 21 nonlocal forces, 22 Bloch H_k application / filter step,
 * 23 Bloch projections; ids < 32. */
sparc_status sparc_gpu_profile(sparc_gpu_ctx ctx, int enable);
sparc_status sparc_gpu_profile_read(sparc_gpu_ctx ctx, int kernel_id, double* total_ms, long* launches);

/* ---- Learned initial density (warm start of the SCF) ----------------------
 * The SCF of Sec. 2.1 starts from a superposition of atomic densities; the
 * warm start replaces that guess by the prediction of a small periodic
 * convolutional network trained on converged densities of related
 * geometries (machine-learning methods are a direction named in Sec. 4).
 *
 * Features: 3 channels f_c(x) = sum over atoms and periodic images within
 * 6 w_c of exp(-|x - R_I - n L|^2 / (2 w_c^2)); d_feat is 3 x N_d float32,
 * channel-major, grid order.  widths: 3 positive host doubles (Bohr). */
sparc_status sparc_gpu_features(sparc_gpu_ctx ctx, const double* widths, float* d_feat);

/* Network: a1 = relu(conv(W1, f) + b1) (3 -> 16), a2 = relu(conv(W2, a1) +
 * b2) (16 -> 16), z = conv(W3, a2) + b3 (16 -> 1), 3x3x3 periodic
 * cross-correlation; rho = N_e softplus(z) / (dV sum softplus(z)).
 * d_w: SPARC_CNN_NPARAMS float32 in the order W1 (16,3,27), b1, W2 (16,16,27),
 * b2, W3 (1,16,27), b3; tap k = 9 (dz+1) + 3 (dy+1) + (dx+1) for neighbour
 * p + (dx, dy, dz).  d_act: caller scratch of 33 N_d float32 that keeps
 * a1, a2, z for the backward pass.  d_rho: N_d float64 output. */
#define SPARC_CNN_NPARAMS 8673
sparc_status sparc_gpu_cnn_forward(sparc_gpu_ctx ctx, const float* d_w, const float* d_feat, float* d_act,
                                   double* d_rho);

/* Gradient of loss = mean_p (rho_p - target_p)^2 with respect to the
 * parameters, from the forward pass's d_act and d_rho (same d_w, d_feat).
 * d_grad: SPARC_CNN_NPARAMS float32 out; d_loss: one device double out (may
 * be NULL).  Deterministic (fixed-order FP64 reductions). */
sparc_status sparc_gpu_cnn_backward(sparc_gpu_ctx ctx, const float* d_w, const float* d_feat, const float* d_act,
                                    const double* d_rho, const double* d_target, float* d_grad, double* d_loss);

/* One Adam step (Kingma & Ba) on n float32 parameters with float32 moments
 * d_m, d_v (start at zero); t >= 1 is the step count for bias correction. */
sparc_status sparc_gpu_adam_step(sparc_gpu_ctx ctx, float* d_w, const float* d_grad, float* d_m, float* d_v, int n,
                                 int t, double lr, double beta1, double beta2, double eps);

/* Initial density for the SCF: the network's prediction with widths
 * (0.5, 1.0, 2.0) Bohr, or the atomic-density guess (sparc_gpu_sad_density)
 * when the prediction is not finite or dV sum |rho - rho_SAD| / N_e >
 * max_l1.  *used_cnn (host, may be NULL) = 1 when the prediction was kept.
 * Synchronises once. */
sparc_status sparc_gpu_warm_start(sparc_gpu_ctx ctx, const float* d_w, double max_l1, double* d_rho, int* used_cnn);

#ifdef __cplusplus
}
#endif

#endif /* SPARC_GPU_H */
