/*
 * pss.h - C ABI of the MI355X (gfx950) parallel square-root iterated smoother.
 *
 * Method: Yaghoobi, Corenflos, Hassan, Sarkka, "Parallel square-root
 * statistical linear regression for inference in nonlinear state space
 * models".  The library computes, on one GPU and for a batch of independent
 * sequences,
 *   - the statistical linear regression of the model around a nominal
 *     trajectory: the generalised SLR (Section 2.3) with a positive-weight
 *     sigma-point rule (cubature, unscented or Gauss-Hermite; Section 4.3),
 *     or the first-order Taylor expansion (Section 4.2),
 *   - the square-root parallel Kalman filter elements (Lemma 1, Tables 1-2)
 *     and their associative scan (Lemma 2, Table 3, Algorithm 1),
 *   - the square-root parallel RTS smoother (Lemmas 3-4, Tables 4-5,
 *     Algorithm 2, a reverse associative scan),
 *   - the iterated posterior linearisation loop (Algorithm 3),
 *   - the pseudo-log-likelihood (Section 5.1, eq. log-likelihood) and its
 *     gradient with respect to the model parameters at a frozen nominal
 *     trajectory (Section 5.2, eq. gradient).
 *
 * Conventions shared by every entry point
 *   - Every buffer pointer is a DEVICE pointer unless its name ends in
 *     "_host".  The caller allocates and owns every buffer; the library never
 *     allocates device memory and keeps no device state between calls.
 *   - Every call is asynchronous on the caller's HIP stream `stream` and
 *     returns PSS_OK or a negative status.  Arguments are validated on the
 *     host before anything is enqueued; a failed validation enqueues nothing.
 *     Numerical breakdown (a NaN) is not a status: it propagates into the
 *     outputs.
 *   - Floating-point buffers hold `dtype` elements (float or double).
 *   - A batch holds B sequences.  Sequence b has n_b = y_off[b+1]-y_off[b] >= 1
 *     measurements y_1..y_n and n_b + 1 states x_0..x_n.  Measurements and
 *     step quantities are indexed by the global STEP SLOT y_off[b] + (k-1)
 *     for step k = 1..n_b (T_y = y_off[B] slots).  State quantities are indexed
 *     by the global STATE SLOT y_off[b] + b + k, k = 0..n_b (T_x = T_y + B).
 *   - Every array is structure-of-arrays, component-major: component c of
 *     slot t is at [c * count + t] where count is T_y or T_x.  Square matrices
 *     are row-major (component i*n + j); lower-triangular factors are packed
 *     row-major (component i*(i+1)/2 + j, j <= i).
 *   - Step slot j of a linearisation holds the transition x_{k-1} -> x_k
 *     (F_{k-1}, c_{k-1}, S_Lambda_{k-1}) together with the measurement model of
 *     y_k (H_k, d_k, S_Omega_k), for the step k it feeds (eq. linear-params).
 *   - Covariances are carried only as lower Cholesky factors with a
 *     non-negative diagonal (the Tria operator of Section 2.2).
 */
#ifndef PSS_H
#define PSS_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define PSS_OK 0
#define PSS_EINVAL (-1)       /* null pointer, bad size, bad offsets, ... */
#define PSS_EUNSUPPORTED (-2) /* dtype / model / dimension not built       */
#define PSS_EWORKSPACE (-3)   /* workspace smaller than pss_workspace_size */
#define PSS_EHIP (-4)         /* HIP launch or runtime error               */

/* ---- enums -------------------------------------------------------------- */
typedef enum { PSS_F32 = 0, PSS_F64 = 1 } pss_dtype;

typedef enum {
    /* affine Gaussian model of eq. linear-model; the caller supplies its
       square-root parameters as a pss_gamma (possibly shared by all steps) */
    PSS_MODEL_LINEAR = 0,
    /* coordinated-turn target with two bearings-only sensors (Section 6.2):
       x = (px, py, vx, vy, w), nx = 5, ny = 2, additive noise with
       Q(theta) = q1 Qv + q2 Qw (integrated white-noise acceleration) and
       R(theta) = sigma^2 I, theta = (log q1, log q2, log sigma). */
    PSS_MODEL_CT_BEARINGS = 1,
    /* stochastic Ricker population model with Poisson counts (Section 6.1):
       nx = ny = 1, x_k = log a + x_{k-1} - exp(x_{k-1}) + q_k, q_k ~ N(0, Q),
       y_k | x_k ~ Poisson(b exp(x_k)); theta = (log a, log b, log Q).  The
       measurement noise is not additive: E[y|x] = V[y|x] = b exp(x), and the
       conditional variance enters S_Omega through E[V[y|x]] (GSLR moments,
       Section 2.3).  The paper's point-mass prior at log c is given as m0 =
       log c with a small factor N0 > 0 (a sigma-point rule regresses on the
       spread of the marginal, so a zero factor has no regression). */
    PSS_MODEL_RICKER_POISSON = 2
} pss_model_kind;

/* linearisation of a nonlinear model (every model but PSS_MODEL_LINEAR).
   The sigma-point rules have positive weights w_i summing to one and unit
   points xi_i; for the marginal N(m, N N^T) the points are m + N xi_i. */
typedef enum {
    /* statistical linear regression with the third-degree cubature rule
       (Section 4.3), 2 nx points +-sqrt(nx) e_i: the iterated posterior-
       linearisation smoother */
    PSS_LIN_CUBATURE = 0,
    /* first-order Taylor expansion at the nominal mean (Section 4.2): the
       iterated extended smoother; S_Lambda and S_Omega are the conditional
       covariance factors at the mean */
    PSS_LIN_TAYLOR = 1,
    /* unscented rule with alpha = 1, beta = 0 and spread kappa = ut_kappa
       (>= 0, so every weight is positive): the centre with weight
       kappa / (nx + kappa) (dropped when kappa = 0) and +-sqrt(nx + kappa) e_i
       with weight 1 / (2 (nx + kappa)) */
    PSS_LIN_UNSCENTED = 2,
    /* tensor-product Gauss-Hermite rule with gh_order points per coordinate
       (gh_order^nx points, at most 1024; gh_order in 2..20) */
    PSS_LIN_GAUSS_HERMITE = 3
} pss_linearization;

/* form of the parallel filter and smoother */
typedef enum {
    /* square-root form (Lemmas 1-4, right columns of Tables 1-5): the
       library's method */
    PSS_FORM_SQRT = 0,
    /* standard covariance form (left columns of Tables 1-5), for comparison;
       honoured by pss_slr_linearize, pss_ipls_iterate, pss_loglik and
       pss_sequential_smoother only.
       The "N" buffers of marginals, the nominal's included (on input and on
       output), then hold the packed lower triangle of the covariance P, not a
       factor; the cubature SLR factors P itself (Cholesky).  The prior is
       still given as a factor N0. */
    PSS_FORM_COV = 1
} pss_form;

/* operations for pss_workspace_size */
typedef enum {
    PSS_OP_SLR = 0,
    PSS_OP_FILTER_ELEMENTS = 1,
    PSS_OP_FILTER_SCAN = 2,
    PSS_OP_SMOOTHER_SCAN = 3,
    PSS_OP_IPLS = 4,
    PSS_OP_LOGLIK = 5,
    PSS_OP_LOGLIK_GRAD = 6,
    PSS_OP_SEQUENTIAL = 7,
    PSS_OP_LOGLIK_GRAD_IFT = 8,
    PSS_OP_LOGLIK_VJP = 9,
    PSS_OP_SCORE_FISHER = 10
} pss_op;

/* ---- problem description (host struct, read during the call only) ----- */
typedef struct pss_problem {
    int32_t model;              /* pss_model_kind                              */
    int32_t dtype;              /* pss_dtype                                   */
    int32_t nx, ny;             /* state / measurement dimension               */
    int32_t B;                  /* number of sequences, >= 1                   */
    const int64_t *y_off;       /* device [B+1], y_off[0] = 0, strictly rising */
    const int64_t *y_off_host;  /* host copy of y_off (launch planning)        */
    const void *m0;             /* device [nx] prior mean, shared by sequences */
    const void *N0;             /* device [nx(nx+1)/2] packed prior factor     */
    /* model constants (ignored by PSS_MODEL_LINEAR) */
    double dt;                  /* CT time step                                */
    double theta[3];            /* CT: log q1, log q2, log sigma;
                                   Ricker: log a, log b, log Q                 */
    double sensors[4];          /* CT: s1x, s1y, s2x, s2y                      */
    /* launch shape overrides (0 = library default / autotuned):
       block threads per scan tile (64, 128 or 256; default 64) and elements
       folded sequentially per thread (>= 1) at the finest level of both
       scans (default 4 for the filter scan, 2 for the smoother scan) */
    int32_t scan_threads;
    int32_t scan_elems;
    /* pss_linearization used by every call that linearises the model
       (slr_linearize, ipls_iterate, loglik, loglik_grad, ipls_batched,
       sequential_smoother); 0 = cubature */
    int32_t linearization;
    /* pss_form; 0 = square root */
    int32_t form;
    /* PSS_LIN_GAUSS_HERMITE: points per coordinate (2..20) */
    int32_t gh_order;
    /* PSS_LIN_UNSCENTED: spread kappa (finite, >= 0) */
    double ut_kappa;
} pss_problem;

/* Square-root linearisation parameters Gamma^sqrt (eq. Gamma-s), SoA over
   step slots.  stride = 1: one set per step slot (arrays of T_y slots);
   stride = 0: a single set shared by every step (arrays of 1 slot).
     F  [nx*nx]  c [nx]  SL [nx(nx+1)/2]   transition, row-major / packed
     H  [ny*nx]  d [ny]  SO [ny(ny+1)/2]   measurement                    */
typedef struct pss_gamma {
    void *F, *c, *SL, *H, *d, *SO;
    int64_t stride;
} pss_gamma;

/* Square-root filter elements Pi^f_k = {A, b, U, eta, Z} (eq. pi-f), SoA over
   step slots: A [nx*nx], b [nx], U [nx(nx+1)/2], eta [nx], Z [nx(nx+1)/2].
   Z is stored as the packed lower factor Tria(Z_k) (same J_k = Z Z^T; this is
   the squaring rule stated in the proof of Lemma 1). */
typedef struct pss_felem {
    void *A, *b, *U, *eta, *Z;
} pss_felem;

/* Checkpoint of the log-likelihood's filter pass, kept between pss_loglik
   (which fills it) and the gradient calls (which consume it) so that the
   backward pass does not repeat the forward filter scan.  Caller-owned
   device memory of pss_ckpt_size(p, level) bytes.  level chooses what is
   stored (level checkpointing of the scan of Algorithm 1):
     0       every filtering marginal (nx + nx(nx+1)/2 numbers per state);
     l >= 1  the exclusive prefixes of the filter scan's level-l elements
             (the filtering marginal before each level-l element: one per
             4 states at level 1, one per 1024 at level 2 with the default
             shapes); the backward pass re-runs only the levels below l;
   a level at or above the scan's top keeps nothing but the per-sequence
   log-likelihoods, and the backward pass re-runs the whole filter scan.
   `tag` is written by pss_loglik and identifies the problem (sizes, model,
   theta, launch shape, level); a gradient call with another problem is
   refused.  The nominal, y and (linear models) Gamma of the gradient call
   must be those of the pss_loglik call that filled it. */
typedef struct pss_ckpt {
    int32_t level;
    void *buf;
    size_t bytes;
    uint64_t tag;
} pss_ckpt;

/* ---- entry points --------------------------------------------------------- */

/* Bytes of workspace `op` needs for this problem (0 if none). Returns 0 and
   sets the last error for an invalid problem. */
size_t pss_workspace_size(const pss_problem *p, int32_t op);

/* Statistical linear regression (Sections 2.3, 4.1-4.3) of a nonlinear model
   around the nominal marginals (m_nom [nx][T_x], N_nom packed [T_x]) with
   the problem's linearisation (a sigma-point rule or the Taylor expansion).
   Transition parameters of slot (b, k) come from the marginal at state k-1,
   measurement parameters from the marginal at state k.  CT bearings are
   taken on the branch nearest to the measurement y (y [ny][T_y]).  The
   regression residual enters the noise factors without a downdate:
   S = Tria([noise columns, sqrt(w_i)(Z_i - zbar - G(X_i - m))]), equal to
   the paper's DownDate(Tria([noise columns, Zx]), G N) because the rules
   integrate second moments exactly; noise columns are the constant factor
   (additive noise) or sqrt(w_i) times the conditional factor at each point
   (Poisson counts).  Writes `out` (stride must be 1).  Nonlinear models
   only. */
int pss_slr_linearize(const pss_problem *p, const void *m_nom, const void *N_nom,
                      const void *y, const pss_gamma *out, hipStream_t stream);

/* Square-root filter elements of Lemma 1 (Table 1 for k = 1, Table 2 for
   k > 1) for every step of every sequence, from the linearisation `g`
   (stride 0 or 1) and the measurements y [ny][T_y].  Writes `out`. */
int pss_sqrt_filter_elements(const pss_problem *p, const pss_gamma *g, const void *y,
                             const pss_felem *out, hipStream_t stream);

/* Algorithm 1: inclusive associative scan of the filter elements with the
   square-root operator of Lemma 2 (Table 3), per sequence.  Writes the
   filtering marginals m_f [nx][T_x] and packed N_f [T_x] (state 0 receives
   the prior).  `el` is read only.  ws: pss_workspace_size(PSS_OP_FILTER_SCAN). */
int pss_sqrt_filter_scan(const pss_problem *p, const pss_felem *el, void *m_f, void *N_f,
                         void *ws, size_t ws_bytes, hipStream_t stream);

/* Algorithm 2: smoother elements of Lemma 3 (Table 4; the last state of each
   sequence takes E = 0, g = m^f_n, D = N^f_n) built from the transition part
   of `g` and the filtering marginals, then the reverse associative scan with
   the operator of Lemma 4 (Table 5).  Writes m_s [nx][T_x], packed N_s.
   ws: pss_workspace_size(PSS_OP_SMOOTHER_SCAN). */
int pss_sqrt_smoother_scan(const pss_problem *p, const pss_gamma *g, const void *m_f,
                           const void *N_f, void *m_s, void *N_s, void *ws, size_t ws_bytes,
                           hipStream_t stream);

/* Algorithm 3: n_iter passes of (SLR at the nominal, filter elements,
   filter scan, smoother scan).  m_nom / N_nom hold the initial nominal on
   entry and the final smoothing marginals on exit.  m_f / N_f (nullable)
   receive the last pass's filtering marginals.  For PSS_MODEL_LINEAR the
   linearisation `g` is used as is on every pass (the SLR of an affine model
   is the model itself); for a nonlinear model `g` must be NULL.
   ws: pss_workspace_size(PSS_OP_IPLS). */
int pss_ipls_iterate(const pss_problem *p, const pss_gamma *g, const void *y, int32_t n_iter,
                     void *m_nom, void *N_nom, void *m_f, void *N_f, void *ws, size_t ws_bytes,
                     hipStream_t stream);

/* Bytes of a checkpoint of this level for this problem (0 and the last
   error set for an invalid problem or a negative level). */
size_t pss_ckpt_size(const pss_problem *p, int32_t level);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the same
   n_iter passes as pss_ipls_iterate, same arguments and outputs, with the
   workspace taken from a file-scope device array of the library instead of
   a caller buffer.  Makes no allocation.  The array holds
   pss_noalloc_max_bytes() bytes (64 MiB: about 4 * 10^4 coordinated-turn
   steps in FP64); a problem whose PSS_OP_IPLS workspace is larger is refused
   with PSS_EWORKSPACE before anything is enqueued.  Each GPU the library
   runs on holds its own copy until the process ends.  Every call on one GPU
   shares that GPU's copy: calls that overlap in time on one GPU (several
   streams or threads) race and give undefined results.  The array keeps the
   last call's contents; nothing in it needs to start at zero. */
size_t pss_noalloc_max_bytes(void);
int pss_ipls_iterate_noalloc(const pss_problem *p, const pss_gamma *g, const void *y,
                             int32_t n_iter, void *m_nom, void *N_nom, void *m_f, void *N_f,
                             hipStream_t stream);

/* Pseudo-log-likelihood of Section 5.1: the model is linearised at the
   nominal (nonlinear models; for LINEAR `g` is used), filtered with
   Algorithm 1, and
   ll[b] = sum_k log N(y_k; H_k m^-_k + d_k, Y_k Y_k^T) with the predicted
   factor Y_k = Tria([H_k Tria([F_{k-1} N^f_{k-1}, S_Lambda]), S_Omega]).
   ll: device double [B] (FP64 accumulation for both dtypes).  ckpt
   (nullable; square-root form): filled for a later gradient call (see
   pss_ckpt).  ws: pss_workspace_size(PSS_OP_LOGLIK). */
int pss_loglik(const pss_problem *p, const pss_gamma *g, const void *m_nom, const void *N_nom,
               const void *y, double *ll, pss_ckpt *ckpt, void *ws, size_t ws_bytes,
               hipStream_t stream);

/* Gradient of the pseudo-log-likelihood with respect to theta = (log q1,
   log q2, log sigma) at a FROZEN nominal (the partial derivative term of
   eq. gradient; PSS_MODEL_CT_BEARINGS only, any linearisation), by a
   hand-written reverse-mode adjoint of the square-root filter pass.  With
   the nominal fixed, theta enters only through S_Lambda and S_Omega.  The
   cotangents of the filtering marginals (Gram cotangents dl/dP, never
   factor cotangents) obey lambda_{k-1} = T_k(lambda_k), an affine map per
   step built from the step's Kalman gain; the maps compose associatively,
   so the VJP of the filter scan runs as a reverse associative scan over the
   same tile levels.  Each step's VJP then gives the Gram cotangents of
   Lambda_k and Omega_k, contracted with dQ/dtheta and dR/dtheta.
   ckpt (nullable): a checkpoint filled by pss_loglik for this problem and
   nominal -- the forward filter pass is then not repeated (level 0) or
   only its levels under the checkpoint are re-run; NULL runs the forward
   pass first.  Outputs (device double): ll [B]; grad [3][B] per sequence,
   component-major (nullable); theta_bar [3] = sum_b ll_bar[b] grad[.][b]
   (nullable; ll_bar nullable means all ones).
   ws: pss_workspace_size(PSS_OP_LOGLIK_GRAD). */
int pss_loglik_grad(const pss_problem *p, const void *m_nom, const void *N_nom, const void *y,
                    const double *ll_bar, const pss_ckpt *ckpt, double *ll, double *grad,
                    double *theta_bar, void *ws, size_t ws_bytes, hipStream_t stream);

/* Vector-Jacobian product of the pseudo-log-likelihood (Section 5.1) with
   respect to the linearisation and the prior, at a frozen nominal, by the
   same reverse-mode adjoint as pss_loglik_grad; any model, square-root
   form.  Outputs, each step's cotangent scaled by its sequence's ll_bar[b]
   (ll_bar nullable: ones):
     g_bar   (stride 1, [.][T_y] in the dtype): the cotangent of every
             field of Gamma at every step slot in the library's
             representation -- F, c, H, d entrywise, S_L and S_O as the
             lower triangles of 2 Lambda_bar S_L and 2 Omega_bar S_O (the
             factor cotangents of the Gram cotangents);
     m0_bar  [nx][B], N0_bar [nx(nx+1)/2][B] (both nullable, together):
             per sequence, the cotangent of the prior mean and of its
             factor (lower triangle of 2 P0_bar N0);
     ll [B]  the log-likelihoods.
   For a linear model with a shared Gamma (stride 0) the gradient is the
   sum of g_bar over the step slots.  ckpt as for pss_loglik_grad.
   ws: pss_workspace_size(PSS_OP_LOGLIK_VJP). */
int pss_loglik_vjp(const pss_problem *p, const pss_gamma *g, const void *m_nom,
                   const void *N_nom, const void *y, const double *ll_bar, const pss_ckpt *ckpt,
                   double *ll, const pss_gamma *g_bar, void *m0_bar, void *N0_bar, void *ws,
                   size_t ws_bytes, hipStream_t stream);

/* The same theta gradient as pss_loglik_grad by another route, kept as a
   cross-check: the sensitivities dl/dLambda_k and dl/dOmega_k as posterior
   expectations of the complete-data score (Fisher's identity), from the
   parallel square-root smoother of the linearised model.  Same outputs as
   pss_loglik_grad without a checkpoint.
   ws: pss_workspace_size(PSS_OP_SCORE_FISHER). */
int pss_score_fisher(const pss_problem *p, const void *m_nom, const void *N_nom, const void *y,
                     const double *ll_bar, double *ll, double *grad, double *theta_bar,
                     void *ws, size_t ws_bytes, hipStream_t stream);

/* Gradient of the pseudo-log-likelihood at the IPLS fixed point (Section
   5.2, eq. implicity_function_theorem, Algorithm 4): the total derivative of
   l(theta) = lhat(theta, n*(theta)) with respect to theta = (log q1, log q2,
   log sigma), where n* = KS(n*, theta) is the nominal that IPLS converges to
   (the caller passes it: m_nom, N_nom in the problem's form, e.g. after
   enough pss_ipls_iterate passes).  The derivative of n* with respect to
   theta solves the linear fixed point dn = (dKS/dn) dn + dKS/dtheta; each
   of the n_iter iterations (>= 1; the error
   contracts like the IPLS iteration itself) is one parallel covariance-form
   pass (SLR, elements, filter scan, smoother scan) evaluated with three
   tangents per number, the value held at n*.  A last tangent pass gives
   the log-likelihood and its total derivative.  PSS_MODEL_CT_BEARINGS,
   FP64 or FP32 (the terms are summed in FP64), any linearisation.  The iteration converges where the IPLS
   iteration itself converges at n* (the operator-norm condition of the
   paper); where IPLS has no fixed point (it can cycle on long bearings-only
   tracks started from the prior) the tangents grow without bound.  Outputs
   (device double): ll [B]; grad [3][B] per sequence, component-major;
   delta [B] (nullable): per sequence, the largest change of the nominal's
   tangents in the last iteration relative to max(1, their size) -- a
   convergence check (infinite once a tangent has overflowed).  ws: pss_workspace_size(PSS_OP_LOGLIK_GRAD_IFT). */
int pss_loglik_grad_ift(const pss_problem *p, const void *m_nom, const void *N_nom,
                        const void *y, int32_t n_iter, double *ll, double *grad, double *delta,
                        void *ws, size_t ws_bytes, hipStream_t stream);

/* Sequential comparator: the same n_iter passes as pss_ipls_iterate, but
   the filter and smoother run as the sequential recursions, walking
   k = 1..n then n-1..0; only the SLR is parallel.  The square-root
   recursions (one wavefront per sequence, each step's Tria rows spread over
   its lanes), or with PSS_FORM_COV the standard Kalman filter and RTS
   smoother (one thread per sequence; marginals then hold P, as in
   pss_ipls_iterate).  Same
   arguments and outputs as pss_ipls_iterate.
   ws: pss_workspace_size(PSS_OP_SEQUENTIAL). */
int pss_sequential_smoother(const pss_problem *p, const pss_gamma *g, const void *y,
                            int32_t n_iter, void *m_nom, void *N_nom, void *m_f, void *N_f,
                            void *ws, size_t ws_bytes, hipStream_t stream);

/* Per-sequence divergence record (the breakdown Section 6.3 counts: a
   non-finite result).  Numerical breakdown is not a status code of the
   entry points -- NaN and infinity propagate into that sequence's outputs
   only, never into another sequence's (no tile spans two sequences).  This
   call ORs marg_bit into status[b] (device int32 [B], caller-cleared) if
   any component of sequence b's marginals (m [nx][T_x], N packed [T_x]:
   filtering or smoothing, the caller says which through its bit, e.g.
   PSS_STATUS_FILTER / PSS_STATUS_SMOOTHER) is NaN or infinite, and ll_bit
   if ll[b] (device double [B]) is.  m, N nullable together; ll nullable;
   not both. */
#define PSS_STATUS_FILTER 1
#define PSS_STATUS_SMOOTHER 2
#define PSS_STATUS_LOGLIK 4
int pss_nan_status(const pss_problem *p, const void *m, const void *N, int32_t marg_bit,
                   const double *ll, int32_t ll_bit, int32_t *status, hipStream_t stream);

/* ---- ragged batches of several model groups in one persistent launch ---- */

/* One model group of a batched call: a ragged batch of sequences of one
   model.  Supported groups: PSS_MODEL_CT_BEARINGS (nx 5, ny 2) with the
   cubature or Taylor linearisation, and PSS_MODEL_LINEAR with nx 4, ny 2
   (e.g. constant velocity).  All groups of a call share the dtype and the
   launch-shape overrides. */
typedef struct pss_group {
    const pss_problem *p;  /* model, dimensions, batch offsets, prior        */
    const pss_gamma *g;    /* linear: its parameters (stride 0/1); CT: NULL  */
    const void *y;         /* [ny][T_y] measurements                         */
    void *m_nom, *N_nom;   /* in: initial nominal; out: after n_iter passes */
} pss_group;

/* Workspace bytes of pss_ipls_batched for these groups (0 if invalid). */
size_t pss_batched_workspace_size(const pss_group *groups, int32_t n_groups);

/* Algorithm 3 for up to 4 groups of ragged sequences, each pass ONE
   persistent kernel launch (plus a flag-clearing kernel): a work queue of
   filter tiles then smoother tiles of every sequence of every group; a tile
   fuses the SLR of Section 4.3 (CT), the elements of Lemma 1 / Table 4, the
   sequential fold, the in-LDS tree and the down-sweep, and chains with its
   neighbour tile (inclusive prefix of tile t = prefix of tile t-1 (x) tile
   aggregate).  Waits only target earlier queue items, are bounded, and set
   bit flags in `status` (device int, nullable; 0 = ok) if a bound is hit.
   Launch shape: the problem's overrides, else the autotuned shape for this
   batch signature (pss_autotune, or the file named by the environment
   variable PSS_TUNE_CACHE), else defaults.  Bitwise reproducible for a
   given shape.  The pass sequence can be captured in a HIP graph. */
int pss_ipls_batched(const pss_group *groups, int32_t n_groups, int32_t n_iter, int32_t *status,
                     void *ws, size_t ws_bytes, hipStream_t stream);

/* Workspace bytes of pss_autotune. */
size_t pss_autotune_workspace_size(const pss_group *groups, int32_t n_groups);

/* Autotuner: times one batched pass for each candidate launch shape (block
   threads 64/128/256, filter and smoother elements per thread 1..8) on the
   caller's data (the nominal is copied, not modified), keeps the fastest for
   this batch signature (dtype, models, batch sizes, log2 of total steps) in a
   host cache used by pss_ipls_batched, and writes the cache to
   cache_path_host if not NULL.  best_host (nullable, 3 ints) receives
   (threads, filter elements, smoother elements).  Synchronises the stream. */
int pss_autotune(const pss_group *groups, int32_t n_groups, void *ws, size_t ws_bytes,
                 const char *cache_path_host, int32_t *best_host, hipStream_t stream);

/* Validation only: returns the status the entry points would return for
   this problem before enqueuing work (no HIP call is made). */
int pss_validate(const pss_problem *p);

/* Message of the last error raised on the calling thread ("" if none). */
const char *pss_last_error(void);

/* Library version string. */
const char *pss_version(void);

/* Instrumentation (not part of the method).  While enabled, every kernel
   launch of the entry points above is bracketed by two HIP events recorded
   on the caller's stream (skipped while that stream is being captured into
   a graph).  Process-wide switch; returns PSS_OK. */
int pss_kernel_timing(int32_t enable);

/* Waits for the events recorded since the last call, then writes one text
   line per (kernel, scan level): "<kernel> <level> <launches> <total ms>\n"
   (kernel = filter_up, filter_top, filter_down, smoother_up, ..., slr,
   filter_elements, loglik_terms, grad_terms, sequential, persistent_pass),
   NUL-terminated and truncated to cap bytes, into buf (host), and clears
   the records.  With buf NULL nothing is written or cleared.  Returns the
   bytes needed (text + NUL), or a negative status. */
int64_t pss_kernel_times(char *buf, size_t cap);

#ifdef __cplusplus
}
#endif

#endif /* PSS_H */
