/*
 * libsignkrylov -- sign(H_W) b for the non-Hermitian Wilson kernel
 * H_W = gamma5 D_W(mu) by restarted multishift FOM with LR deflation
 * (Bloch, Breu, Frommer, Heybrock, Schaefer, Wettig, "Krylov subspace
 * methods and the sign function: multishifts and deflation in the
 * non-Hermitian case", Lattice 2009; Algorithm 1, restarted FOM-LR(m,k)).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All vector, matrix and link buffers are DEVICE memory owned by the
 *   caller.  The library never frees them and allocates no device memory
 *   itself; scratch space is the caller's `ws` workspace, sized by the
 *   matching *_workspace_bytes query.  Small parameter arrays marked
 *   "host" are read before the call returns.
 * - Every call is ordered on `stream` (0 = the null stream).  Calls that
 *   report results on the host (k_done, sk_stats) synchronise `stream`.
 * - Complex numbers are interleaved (re, im): 16 bytes for SK_C128
 *   (double), 8 bytes for SK_C64 (float).
 * - Lattice: dims = (Lx, Ly, Lz, Lt), V = Lx*Ly*Lz*Lt, site index
 *   s = ((t*Lz + z)*Ly + y)*Lx + x; direction 0..3 = x, y, z, t.
 *   Spinor fields are component-major: element (c, s) at c*V + s with
 *   c = 3*spin + colour (12 components), n = 12 V.  Links are
 *   [4][3][3][V]: U_nu(x)_{ab} at ((nu*3 + a)*3 + b)*V + s.
 * - The operator (paper Sect. 1, defined there by reference) is
 *     D_W(mu) psi(x) = psi(x) - kappa sum_nu [ e^{+mu d_nu,t} (1 - gamma_nu) U_nu(x) psi(x+nu)
 *                                         + e^{-mu d_nu,t} (1 + gamma_nu) U_nu(x-nu)^+ psi(x-nu) ],
 *   H_W = gamma5 D_W, chiral basis (gamma5 = diag(1,1,-1,-1)),
 *   periodic in space, antiperiodic in time when t_antiperiodic != 0.
 *   H_W(mu)^H = H_W(-mu).
 * - Return value: SK_OK (0) or a negative sk_status.  Arguments are
 *   checked on the host before any launch; on error nothing is launched
 *   and sk_last_error() returns a message (thread-local).  No exception
 *   crosses this interface.
 */
#ifndef SIGNKRYLOV_H
#define SIGNKRYLOV_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SK_OK = 0,
  SK_ERR_ARG = -1,       /* invalid argument: sizes, null pointers, aliasing */
  SK_ERR_HIP = -2,       /* a HIP runtime call failed */
  SK_ERR_NOCONV = -3,    /* max_cycles reached; x holds the last iterate */
  SK_ERR_SINGULAR = -4,  /* H_k - sigma_i singular: FOM iterate undefined */
  SK_ERR_NAN = -5,       /* non-finite value in the input or the iteration */
  SK_ERR_WORKSPACE = -6  /* workspace smaller than the query returned */
} sk_status;

typedef enum {
  SK_C128 = 0,   /* complex double storage and arithmetic */
  SK_C64 = 1     /* complex float storage; reductions accumulate in double */
} sk_dtype;

typedef enum {
  SK_METHOD_FOM = 0,    /* restarted multishift FOM, collinear residuals (Algorithm 1) */
  SK_METHOD_GMRES = 1   /* restarted multishift GMRES (Sect. 2, 3, 5: GMRES-LR) */
} sk_method;

typedef enum {
  SK_PREC_FP64 = 0,   /* every vector in complex double */
  SK_PREC_MIXED = 1   /* complex-float basis and stencil, double refinement */
} sk_precision;

typedef struct {
  int32_t dims[4];          /* Lx, Ly, Lz, Lt, each >= 1 */
  int32_t t_antiperiodic;   /* 1: antiperiodic time boundary, 0: periodic */
  double kappa;             /* hopping parameter, 1/(2 m_W + 8) */
  double mu;                /* quark chemical potential (time hops) */
  const void* links;        /* device, complex double [4][3][3][V] */
  const void* links_c64;    /* device, complex float copy; needed by SK_C64 calls */
} sk_operator;

/*
 * Poles and weights of the Kenney-Laub rational approximation of sign
 * (Sect. 6): g_s(c t) = c t sum_{i=1..s} w_i / (c^2 t^2 + tau_i^2),
 * theta_i = pi (i - 1/2) / (2 s), tau_i = tan(theta_i), w_i = 1/(s cos^2 theta_i),
 * split into N = 2 s first-order terms of eq. (g):
 *   sigma_{2i} = +i tau_i / c,  sigma_{2i+1} = -i tau_i / c,  omega = w_i / (2 c).
 * sigma, omega: host, 2 s complex (re, im interleaved) each.  s in [1, 32], c > 0.
 */
int kl_poles(int s, double c, double* sigma, double* omega);

/* links_c64 = links rounded to complex float (device, 36 V entries each;
   the operator's links_c64 for the complex-float stencil). */
int sk_links_to_c64(const double* links, float* links_c64, int64_t V, hipStream_t stream);

/* Number of lattice sites of an operator (0 if dims are invalid). */
int64_t sk_volume(const sk_operator* op);

/* Thread-local message for the last failing call on this thread. */
const char* sk_last_error(void);

/*
 * w = H_W v  (adjoint = 0)  or  w = H_W^H v = H_W(-mu) v  (adjoint = 1).
 * The matrix-vector product every Krylov step needs (Sect. 2: Krylov
 * methods touch A only through products with vectors).
 * in, out: device, n = 12 V complex of `dtype`; must not overlap.
 */
int wilson_apply(const sk_operator* op, sk_dtype dtype, const void* in, void* out,
                 int adjoint, hipStream_t stream);

/*
 * One cycle of k Arnoldi steps (Sect. 2, Arnoldi relation
 * A V_k = V_k H_k + h_{k+1,k} v_{k+1} e_k^T), with classical Gram-Schmidt
 * applied twice per step (CGS2).
 *   V:  device, (k+1) vectors of n complex `dtype`, vector j at V + j*n.
 *       On entry V[0] holds a nonzero start vector (it is normalised);
 *       on exit V[0..k_done] are orthonormal.
 *   H:  device, complex double, (k+1) x k column-major (ld = k+1);
 *       entries below the subdiagonal are zero.
 *   k_done: host out; k, or the step j < k at which h_{j+1,j} fell below
 *       1e-12 ||A v_j|| (lucky breakdown: K_j is invariant).
 *   ws: device workspace of arnoldi_cycle_workspace_bytes(op, k) bytes.
 * Synchronises `stream` (k_done is read back).
 */
size_t arnoldi_cycle_workspace_bytes(const sk_operator* op, int k);
int arnoldi_cycle(const sk_operator* op, sk_dtype dtype, void* V, double* H, int k,
                  int* k_done, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * The per-cycle multishift FOM step of Algorithm 1 (Sect. 3 and 5):
 *   y_i  = beta rho_i (H_k - sigma_i I)^{-1} e_1,  i = 1..npoles  (double)
 *   x   += V_k sum_i omega_i y_i
 *   X_i += V_k y_i                      (only if X_shift != NULL)
 *   rho_i <- -h_{k+1,k} e_k^T y_i       (collinear residuals r_i = rho_i v_{k+1})
 *   H, beta, rho: device, complex double (H as in arnoldi_cycle, ld = k+1;
 *        beta is one real double; rho has npoles complex entries, in/out).
 *   sigma, omega: host, npoles complex double each (re, im interleaved).
 *   V: device, k orthonormal vectors of `dtype` (vector j at V + j*n).
 *   x, X_shift: device complex double, n and npoles*n entries.
 *   upd_norm: host double out, ||sum_i omega_i y_i||_2.
 *   ws: device workspace of multishift_fom_restart_workspace_bytes(k, npoles).
 * Returns SK_ERR_SINGULAR if some H_k - sigma_i had a zero pivot.
 * Synchronises `stream`.
 */
size_t multishift_fom_restart_workspace_bytes(int k, int npoles);
int multishift_fom_restart(int k, int64_t n, sk_dtype dtype, const double* H,
                           int npoles, const double* sigma, const double* omega,
                           const double* beta, double* rho, const void* V, double* x,
                           double* X_shift, double* upd_norm, void* ws, size_t ws_bytes,
                           hipStream_t stream);

/*
 * LR deflation (Sect. 4): with P = R L^H (L^H R = I_m),
 *   coeff = L^H in                         (device, m complex double)
 *   r_out = (I - P) in
 *   xp_out = R F coeff   (if xp_out and F are non-NULL; F = f(Lambda) in
 *                         the basis R, m x m complex double column-major,
 *                         device; diagonal sign(Re lambda) for LR vectors)
 * R, L: device complex double, m vectors of n entries (vector i at +i*n).
 * in, r_out, xp_out: device complex double, n entries; r_out may equal in,
 * xp_out must not overlap either.
 * ws: device workspace of deflate_project_workspace_bytes(m, n).
 */
size_t deflate_project_workspace_bytes(int m, int64_t n);
int deflate_project(int m, int64_t n, const double* R, const double* L, const double* F,
                    const double* in, double* r_out, double* xp_out, double* coeff,
                    void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * deflate_project without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results as
 * deflate_project; the scratch lives in a 7 MiB device array inside the
 * library, one per GPU, held until the process ends.  Limits: m <= 128 and
 * n <= 12 * 16^4 (larger sizes return SK_ERR_ARG before any launch).  The
 * call allocates nothing.  Every call on one GPU uses that GPU's array:
 * calls that overlap in time on one GPU (other streams, other threads)
 * race and must be serialised by the caller.
 */
int deflate_project_noalloc(int m, int64_t n, const double* R, const double* L, const double* F,
                            const double* in, double* r_out, double* xp_out, double* coeff,
                            hipStream_t stream);

typedef struct {
  int32_t npoles;           /* N first-order poles of eq. (g) */
  const double* sigma;      /* host, N complex (re, im) */
  const double* omega;      /* host, N complex (re, im) */
  int32_t k;                /* restart length k_max (1 <= k <= 256) */
  int32_t max_cycles;       /* cap on restart cycles */
  double tol;               /* stop when ||update|| <= tol*||x|| twice in a row */
  int32_t m;                /* deflation dimension (0: none) */
  const double* R;          /* device, m x n complex double (right vectors) */
  const double* L;          /* device, m x n complex double (left vectors, L^H R = I) */
  const double* F;          /* device, m x m complex double, f(Lambda) in basis R */
  int32_t project_each_cycle; /* 1: projection step after every cycle (Alg. 1) */
  int32_t precision;        /* sk_precision */
  double mixed_switch;      /* SK_PREC_MIXED: cycles run in complex double until the
                               relative update ||sum omega_i y_i|| / ||x|| falls
                               below this, then in complex float (complex-float
                               rounding then only touches the small remaining
                               error).  0 = 1e-3; >= 1 = complex float throughout. */
  double* X_shift;          /* device, N x n complex double, or NULL: per-shift
                               solutions of (A - sigma_i) X_i = (I - P) b */
  int32_t method;           /* SK_METHOD_FOM (Algorithm 1, FOM-LR) or SK_METHOD_GMRES
                               (GMRES-LR: restarted multishift GMRES, see sign_apply) */
  int32_t seed;             /* GMRES-LR: index of the pole whose system is solved by
                               GMRES (-1: the pole nearest the origin) */
  double resid_tol;         /* SK_PREC_MIXED: the FP64 check of the result (see
                               sign_apply) accepts shift i when its true residual
                               ||(I-P)b - (A - sigma_i) X_i|| <= 10 |rho_i| +
                               resid_tol ||(I-P)b||.  0 = 100 tol. */
} sk_sign_params;

/* Kernel classes of a solve, for the optional per-kernel timing. */
typedef enum {
  SK_K_STENCIL = 0,     /* z = H_W u */
  SK_K_GS_DOT = 1,      /* Gram-Schmidt dots V_j^H [u z], u^H u, u^H z (one kernel) */
  SK_K_GS_UPD_DOT = 2,  /* v_j and the next first-pass vector from one pass over V_j */
  SK_K_GS_UPD_NORM = 3, /* final second pass of the last vector (dots + update) */
  SK_K_SMALL = 4,       /* shifted Hessenberg solves */
  SK_K_SOL_UPDATE = 5,  /* x += V_k u (and per-shift X) */
  SK_K_PROJECT = 6,     /* deflation projection / restart vector */
  SK_K_GS_REDUCE = 7,   /* folding of the dot partial sums (large n only) */
  SK_K_COUNT = 8
} sk_kernel_class;

/* Per-class kernel time (HIP events on the call's stream, summed over the
   solve) and algorithmic bytes: the bytes the operation must move at
   minimum (each operand read once, each result written once). */
typedef struct {
  double ms[8];
  double bytes[8];
  int64_t launches[8];
} sk_kernel_times;

typedef struct {
  int32_t cycles;           /* restart cycles run */
  int32_t cycles_c64;       /* of which with the complex-float basis */
  int32_t matvecs;          /* H_W applications (all precisions) */
  int32_t converged;        /* 1 if the stopping rule was met */
  int32_t breakdown;        /* 1 if a cycle ended in lucky breakdown */
  double final_update_norm; /* ||sum omega_i y_i|| of the last cycle */
  double x_norm;            /* ||x|| at exit */
  double* hist_update;      /* host, nullable: per-cycle update norms */
  double* hist_beta;        /* host, nullable: per-cycle ||r|| */
  double* hist_leak;        /* host, nullable: per-cycle ||L^H r|| before projection */
  int32_t hist_cap;         /* capacity of the history arrays */
  sk_kernel_times* times;   /* host, nullable: if set, every kernel of the solve
                               is bracketed by HIP events (slightly slower) */
  double* hist_rho;         /* host, nullable: per cycle the npoles collinearity
                               factors |rho_i| (the norms of the shifted residuals
                               r_i = rho_i (I-P) v_{k+1} the iteration carries),
                               hist_cap rows of npoles doubles */
  double* shift_resid;      /* host, nullable: npoles entries, the FP64 true
                               residuals ||(I-P)b - (A - sigma_i) X_i|| / ||(I-P)b||
                               at exit (filled when per-shift solutions are kept:
                               X_shift given, or mixed precision) */
  double* shift_resid_implicit; /* host, nullable: npoles entries, |rho_i| / ||(I-P)b||
                               at exit, to compare with shift_resid */
  int32_t resid_checked;    /* 1 if shift_resid was computed */
  int32_t resid_ok;         /* 1 if every shift passed the FP64 check */
  double seconds;           /* host wall-clock time of the call */
} sk_stats;

/*
 * x = sign(H_W) b approximated by Algorithm 1 (restarted FOM-LR(m,k)):
 *   x = R F L^H b + sum_i omega_i x_i,  (H_W - sigma_i) x_i = (I - R L^H) b,
 * to the stopping rule above.  b, x: device complex double, n entries,
 * no overlap.  stats: host, nullable.  One host read-back per cycle.
 * Returns SK_ERR_NOCONV if max_cycles ran out (x holds the iterate).
 *
 * GMRES-LR (p->method = SK_METHOD_GMRES, complex double): the same cycles
 * of k Arnoldi steps and projection step, but the seed system s solves the
 * least-squares problem min || beta rho_s e_1 - (Hbar_k - sigma_s I~) y ||
 * (GMRES), with residual V_{k+1} z, and every other system keeps its
 * residual collinear with the seed's by solving the (k+1)-square system
 * [Hbar_k - sigma_i I~, z] [y_i; rho_i'] = beta rho_i e_1; the next cycle
 * starts from (I - P) V_{k+1} z.  These small problems (O(N k^2)) are solved
 * on the host in FP64 from the H read back once per cycle.  Same stopping
 * and divergence rules as FOM-LR.
 *
 * Mixed precision keeps the per-shift solutions X_i (in X_shift, or in the
 * workspace) and, once the stopping rule is met, checks the result in FP64:
 * N complex-double stencil applications give the true residuals
 * (I-P)b - (A - sigma_i) X_i, which must stay within 10 |rho_i| (the
 * residual the iteration carries for shift i) + resid_tol ||(I-P)b||;
 * otherwise the call returns SK_ERR_NOCONV (x holds the iterate and
 * stats->shift_resid the residuals).
 */
size_t sign_apply_workspace_bytes(const sk_operator* op, const sk_sign_params* p);
int sign_apply(const sk_operator* op, const sk_sign_params* p, const double* b, double* x,
               sk_stats* stats, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Gradient of F = Re <eta, g(H_W) b>, g = sum_j omega_j / (x - sigma_j)
 * (no deflation, p->m must be 0; complex double), with respect to the
 * links, U_nu(x) -> exp(i theta^a lambda_a / 2) U_nu(x) at theta = 0, and to mu:
 *   dF = -Re sum_j omega_j z_j^H (dH_W) x_j,
 *   x_j = (H_W - sigma_j)^{-1} b,  z_j = (H_W^H - conj sigma_j)^{-1} eta,
 * the z_j from the same restarted multishift FOM on H_W^H = H_W(-mu).
 *   x_out: device, n complex double, nullable: g(H_W) b (the forward result)
 *   grad_theta: device, double [4][V][8] (direction nu, site, generator a)
 *   grad_mu: host, one double.
 *   stats: host, nullable, two entries (forward solve, adjoint solve).
 * ws: sign_apply_backward_workspace_bytes (holds both sets of per-shift
 * solutions, 2 N n complex doubles).
 */
size_t sign_apply_backward_workspace_bytes(const sk_operator* op, const sk_sign_params* p);
int sign_apply_backward(const sk_operator* op, const sk_sign_params* p, const double* b,
                        const double* eta, double* x_out, double* grad_theta, double* grad_mu,
                        sk_stats* stats, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Algorithm 1 for nsys independent systems at once (many sources, possibly
 * on several gauge fields and lattice sizes), stepped in lockstep: every
 * kernel of a restart cycle is one launch for the whole batch, systems
 * that share a gauge field (same links pointers, dims, kappa, mu, boundary)
 * share each link load in the stencil, finished systems drop out, and a
 * cycle is replayed from a captured HIP graph.  Each system follows the
 * same iteration as sign_apply with the same parameters (same Arnoldi and
 * small-solve arithmetic; the reductions of ||x|| and L^H v are summed in
 * another order, so results agree to rounding, not bit for bit).
 */
typedef struct {
  sk_operator op;           /* this system's operator (by value) */
  const double* b;          /* device, 12 V complex double; may be shared */
  double* x;                /* device, 12 V complex double; overlaps nothing */
  int32_t k;                /* restart length (0: p->k) */
  int32_t m;                /* deflation dimension (0: none) */
  const double* R;          /* device, as in sk_sign_params (m > 0) */
  const double* L;
  const double* F;
  const double* sigma;      /* host, npoles complex, nullable: p->sigma (each
                               lattice may need its own pole scale c) */
  const double* omega;      /* host, nullable: p->omega */
} sk_batch_system;

/*
 * p: npoles, max_cycles, tol, precision, mixed_switch, project_each_cycle
 *   and the default k, sigma, omega shared by all systems; p->m, R, L, F
 *   are ignored; X_shift must be NULL.  SK_PREC_MIXED switches the whole
 *   batch to the complex-float basis once every active system meets the
 *   switch rule.
 * stats: host, nullable, nsys entries.  If stats[0].times is set, the
 *   cycles run as plain launches stamped by HIP events (slower; the same
 *   results bit for bit) and stats[0].times receives, per launch class,
 *   the time and the algorithmic bytes of the systems live in each cycle;
 *   the times of the other entries are not filled.
 * Returns SK_OK if every system converged, else the status of a failing
 * one (every x still holds its iterate; stats[z].converged says which).
 * Workspace: sign_apply_batched_workspace_bytes (0 = invalid arguments).
 */
size_t sign_apply_batched_workspace_bytes(int nsys, const sk_batch_system* sys,
                                          const sk_sign_params* p);
int sign_apply_batched(int nsys, const sk_batch_system* sys, const sk_sign_params* p,
                       sk_stats* stats, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Launch shapes the batched solver's tuner chose for the calling thread's
 * last sign_apply_batched call: rows per thread of the Gram-Schmidt dot
 * kernel and of the update kernel, and right-hand sides per stencil block.
 * The tuner times every candidate on the first call for a batch shape
 * (number and sizes of the systems, their k, precision) and caches the
 * fastest for the life of the process.  Host only; SK_ERR_ARG for NULL.
 */
int sk_batched_last_tile(int* rows_per_thread_dot, int* rows_per_thread_update, int* rhs_per_block);
/* Fix the shapes of later batched calls (process-wide; 1..8 rows per thread
 * each, 1..64 right-hand sides per block), or hand them back to the tuner
 * with (0, 0, 0).  Host only. */
int sk_batched_set_tile(int rows_per_thread_dot, int rows_per_thread_update, int rhs_per_block);

/*
 * Deflation data for Algorithm 1: the m "critical" eigenvalues of H_W
 * (Sect. 4 -- the paper takes R_m, L_m, Lambda_m as given inputs).
 * Krylov-Schur (thick-restart Arnoldi) on A^2 for its eigenvalues of
 * smallest real part finds the eigenvalues of A nearest zero (their squares
 * sit at the left edge of the spectrum of A^2); m + nev_extra of them are
 * computed so the selection can be certified (every |lambda| <= the m-th
 * selected one must be among them).  The same on A^H = H_W(-mu) gives the
 * left invariant subspace.  Output, in an orthonormal Schur basis of the
 * right invariant subspace (an oblique projector equal to the LR one):
 *   R (device, m x n complex double): orthonormal, A R = R T_m;
 *   L (device, m x n complex double): L^H R = I, L^H A = T_m L^H;
 *   F (device, m x m complex double, column-major): sign(T_m) (Newton);
 *   lambda (host, m complex): diag(T_m), sorted by the selection key.
 * P = R L^H and x_P = R F L^H b are exactly the R_m f(Lambda_m) L_m^H of
 * Sect. 4.  The small dense problems (Schur forms, sorting, sign) run in
 * FP64 on the host inside the library.
 */
typedef struct {
  int32_t m;             /* eigenpairs to deflate, 1..128 */
  int32_t nev_extra;     /* extra Ritz pairs computed to certify the selection */
  int32_t ncv;           /* Krylov-Schur basis size (0: automatic) */
  int32_t key;           /* 0: smallest |lambda|, 1: smallest |Re lambda| */
  double tol;            /* relative residual of the converged A^2 Schur vectors */
  int32_t max_restarts;
  int32_t keep;          /* Schur vectors kept at a thick restart, m + nev_extra ..
                            ncv - 8 (0: automatic, halfway between the two) */
} sk_eig_params;

typedef struct {
  int32_t converged;
  int32_t restarts[2];   /* right, left */
  int64_t matvecs;       /* H_W applications */
  double resid[2];       /* largest relative A^2 Schur residual, right / left */
  double gap;            /* key gap between the m-th and (m+1)-th eigenvalue */
  double key_window;     /* largest Re(lambda^2) computed (certification) */
} sk_eig_stats;

size_t deflation_eigensolve_workspace_bytes(const sk_operator* op, const sk_eig_params* p);
int deflation_eigensolve(const sk_operator* op, const sk_eig_params* p, double* R, double* L,
                         double* F, double* lambda, sk_eig_stats* stats, void* ws,
                         size_t ws_bytes, hipStream_t stream);

/*
 * The direct projection methods Sect. 6 compares FOM-LR with (eq. (direct)):
 *   x_k = x_P + ||(I - P) b|| V_k sign(M_k) e_1,   x_P = R F L^H b,
 * no rational approximation and no restarts.
 *   method 0: M_k = H_k from k Arnoldi steps (CGS2) on A from (I - P) b;
 *   method 1: M_k = T_k, the tridiagonal matrix of k two-sided Lanczos
 *             steps (biorthogonal right/left bases of A and A^H = H_W(-mu),
 *             left start (I - L R^H) v_1; "2sL" of Fig. 1).  Serious
 *             breakdown (w^H v = 0) returns SK_ERR_SINGULAR.
 * sign(M_k) by Roberts' method (Newton X <- (X + X^{-1})/2, determinantal
 * scaling while far from convergence), in FP64 on the device.  Fewer than
 * k steps are taken when the Krylov space becomes invariant (the result is
 * then exact up to the deflated part).
 *   k: 1..256;  m, R, L, F as in sk_sign_params (m = 0: no deflation);
 *   b, x: device complex double, n entries, no overlap;
 *   S: device, nullable: on exit sign(M_kk), kk x kk column-major;
 *   stats: host, nullable.
 * Returns SK_ERR_NOCONV if the Newton iteration did not converge in 100
 * steps, SK_ERR_SINGULAR if an iterate was singular.  Complex double.
 */
typedef struct {
  int32_t k_done;        /* Krylov steps taken */
  int32_t breakdown;     /* 1 if the space became invariant before k */
  int32_t newton_iters;  /* Newton iterations for sign(M_kk) */
  int32_t pad;
  double newton_change;  /* relative change of the last Newton iteration */
  double seconds;        /* host wall-clock time of the call */
} sk_direct_stats;

size_t direct_sign_workspace_bytes(const sk_operator* op, int method, int k, int m);
int direct_sign_apply(const sk_operator* op, int method, int k, int m, const double* R,
                      const double* L, const double* F, const double* b, double* x, double* S,
                      sk_direct_stats* stats, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * The overlap Dirac operator at chemical potential mu (Sect. 1; the paper
 * defines it by reference, here in the usual normalisation):
 *   D(m) = (1 - m/2) (1 + gamma5 sign(H_W)) + m      (massless at m = 0),
 * with sign(H_W) v computed by sign_apply(op, p, v) -- Algorithm 1 with the
 * poles, restart length, deflation and precision of p (p->X_shift must be
 * NULL).  gamma5 = diag(1, 1, -1, -1): components 6..11 of a field.
 *   overlap_apply: y = D(m) b.  Workspace overlap_workspace_bytes(op, p, 0).
 *   overlap_solve: x with D(m) x = b by restarted GMRES(k_outer) (classical
 *     Gram-Schmidt twice, Givens least squares on the host), every operator
 *     application one sign_apply; stops when the true relative residual
 *     ||b - D x|| / ||b|| <= 10 tol_outer after the GMRES estimate fell below
 *     tol_outer, else SK_ERR_NOCONV after max_outer applications.  The inner
 *     tolerance p->tol must be well below tol_outer.  Workspace
 *     overlap_workspace_bytes(op, p, k_outer), k_outer in [1, 256].
 * b, y, x: device complex double, n entries, no overlap.  Errors of the inner
 * sign_apply are returned as they are (with its message).
 */
typedef struct {
  int32_t outer_iters;    /* operator applications inside GMRES cycles */
  int32_t restarts;       /* GMRES cycles */
  int64_t sign_calls;     /* sign_apply calls (including true residuals) */
  int64_t inner_matvecs;  /* H_W applications of all inner solves */
  double rel_residual;    /* last true (or estimated) relative residual */
  int32_t converged;
  int32_t pad;
  double seconds;         /* host wall-clock time of the call */
} sk_overlap_stats;

size_t overlap_workspace_bytes(const sk_operator* op, const sk_sign_params* p, int k_outer);
int overlap_apply(const sk_operator* op, const sk_sign_params* p, double mass, const double* b,
                  double* y, sk_stats* stats, void* ws, size_t ws_bytes, hipStream_t stream);
int overlap_solve(const sk_operator* op, const sk_sign_params* p, double mass, int k_outer,
                  int max_outer, double tol_outer, const double* b, double* x,
                  sk_overlap_stats* stats, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Host helpers exposing the library's small dense FP64 routines (used by the
 * eigensolver), column-major complex (re, im) arrays, host memory:
 *   sk_dense_schur: A (n x n) = Q T Q^H, T upper triangular, with the
 *     `count` eigenvalues of smallest key first (key 0: Re, 1: |.|, 2: |Re|).
 *   sk_dense_sign: S = sign(A) by Newton's iteration (Roberts' method).
 * Return SK_OK, or SK_ERR_NOCONV / SK_ERR_SINGULAR.
 */
int sk_dense_schur(int n, const double* A, double* T, double* Q, int key, int count);
int sk_dense_sign(int n, const double* A, double* S);

#ifdef __cplusplus
}
#endif

#endif /* SIGNKRYLOV_H */
