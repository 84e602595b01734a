/*
 * FP64 CPU oracle for the parallel square-root iterated smoother
 * (Yaghoobi, Corenflos, Hassan, Sarkka: "Parallel square-root statistical
 * linear regression for inference in nonlinear state space models").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference against
 * which the HIP library is checked.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no source with
 * the HIP library: its triangularisation uses Givens rotations (the library
 * uses Householder reflections), and its models, SLR, filters and smoothers
 * are written here from the paper independently.
 *
 * Conventions
 *   - every matrix is dense row-major double; a "lower factor" is an n x n
 *     row-major array whose strict upper triangle is zero;
 *   - a sequence has states k = 0..n and measurements y_1..y_n;
 *   - linearisation parameters are stored per step slot j = 0..n-1: slot j
 *     holds the transition (F_j, c_j, S_Lambda_j) that maps x_j to x_{j+1}
 *     and the measurement (H_{j+1}, d_{j+1}, S_Omega_{j+1}) of y_{j+1};
 *   - gamma_stride is 1 for per-step parameters and 0 for one set shared by
 *     every step (time-invariant linear models).
 *
 * Parity status (also stated in the design notes):
 *   - tria, downdate, cubature SLR, filters, smoothers, log-likelihood and
 *     score are pinned by the CPU tests (closed forms, brute force, finite
 *     differences, library routines);
 *   - the first-order Taylor linearisation (iterated extended smoother) is
 *     pinned by finite differences of the model functions and by the
 *     cubature SLR's small-covariance limit;
 *   - the general sigma-point rules (cubature, unscented, Gauss-Hermite) and
 *     the generalised SLR with state-dependent conditional covariance are
 *     pinned by moment exactness, the textbook special cases of the
 *     unscented rule, exactness on affine maps, the printed DownDate form,
 *     and, on the Ricker-Poisson model, by the closed-form lognormal moments
 *     (high-order Gauss-Hermite), finite differences (Taylor) and the
 *     small-spread limit;
 *   - the CT iterated smoother's output values have no printed reference in
 *     the paper: beyond the invariants tested, parity unpinned; the same
 *     holds for the Ricker iterated smoother's outputs.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXD 16 /* largest dimension handled by the fixed-size scratch */

/* ------------------------------------------------------------------------ */
/* small dense helpers                                                      */
/* ------------------------------------------------------------------------ */

/* C (r x c) = A (r x k) * B (k x c) */
static void mat_mul(int r, int k, int c, const double *A, const double *B, double *C)
{
    double tmp[OR_MAXD * OR_MAXD * 4];
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < c; ++j) {
            double s = 0.0;
            for (int t = 0; t < k; ++t)
                s += A[i * k + t] * B[t * c + j];
            tmp[i * c + j] = s;
        }
    memcpy(C, tmp, sizeof(double) * (size_t)(r * c));
}

/* C (r x c) = A^T B with A (k x r), B (k x c) */
static void mat_tmul(int r, int k, int c, const double *A, const double *B, double *C)
{
    double tmp[OR_MAXD * OR_MAXD * 4];
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < c; ++j) {
            double s = 0.0;
            for (int t = 0; t < k; ++t)
                s += A[t * r + i] * B[t * c + j];
            tmp[i * c + j] = s;
        }
    memcpy(C, tmp, sizeof(double) * (size_t)(r * c));
}

/* C (r x c) = A B^T with A (r x k), B (c x k) */
static void mat_mult(int r, int k, int c, const double *A, const double *B, double *C)
{
    double tmp[OR_MAXD * OR_MAXD * 4];
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < c; ++j) {
            double s = 0.0;
            for (int t = 0; t < k; ++t)
                s += A[i * k + t] * B[j * k + t];
            tmp[i * c + j] = s;
        }
    memcpy(C, tmp, sizeof(double) * (size_t)(r * c));
}

static void mat_transpose(int r, int c, const double *A, double *At)
{
    double tmp[OR_MAXD * OR_MAXD * 4];
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < c; ++j)
            tmp[j * r + i] = A[i * c + j];
    memcpy(At, tmp, sizeof(double) * (size_t)(r * c));
}

static void mat_vec(int r, int c, const double *A, const double *x, double *y)
{
    double tmp[OR_MAXD * 2];
    for (int i = 0; i < r; ++i) {
        double s = 0.0;
        for (int j = 0; j < c; ++j)
            s += A[i * c + j] * x[j];
        tmp[i] = s;
    }
    memcpy(y, tmp, sizeof(double) * (size_t)r);
}

static void mat_tvec(int r, int c, const double *A, const double *x, double *y)
{ /* y (c) = A^T x, A r x c */
    double tmp[OR_MAXD * 2];
    for (int j = 0; j < c; ++j) {
        double s = 0.0;
        for (int i = 0; i < r; ++i)
            s += A[i * c + j] * x[i];
        tmp[j] = s;
    }
    memcpy(y, tmp, sizeof(double) * (size_t)c);
}

static void eye(int n, double *I)
{
    for (int i = 0; i < n * n; ++i)
        I[i] = 0.0;
    for (int i = 0; i < n; ++i)
        I[i * n + i] = 1.0;
}

/* Solve L X = B for X, L lower n x n, B n x m (in place allowed). */
static void solve_lower(int n, const double *L, int m, const double *B, double *X)
{
    double tmp[OR_MAXD * OR_MAXD * 4];
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < n; ++i) {
            double s = B[i * m + j];
            for (int t = 0; t < i; ++t)
                s -= L[i * n + t] * tmp[t * m + j];
            tmp[i * m + j] = s / L[i * n + i];
        }
    memcpy(X, tmp, sizeof(double) * (size_t)(n * m));
}

/* Solve L^T X = B for X, L lower n x n, B n x m. */
static void solve_lower_t(int n, const double *L, int m, const double *B, double *X)
{
    double tmp[OR_MAXD * OR_MAXD * 4];
    for (int j = 0; j < m; ++j)
        for (int i = n - 1; i >= 0; --i) {
            double s = B[i * m + j];
            for (int t = i + 1; t < n; ++t)
                s -= L[t * n + i] * tmp[t * m + j];
            tmp[i * m + j] = s / L[i * n + i];
        }
    memcpy(X, tmp, sizeof(double) * (size_t)(n * m));
}

/* X = B L^{-1}  (B r x n, L lower n x n): solve X L = B, i.e. L^T X^T = B^T */
static void right_solve_lower(int r, int n, const double *B, const double *L, double *X)
{
    double Bt[OR_MAXD * OR_MAXD * 4], Xt[OR_MAXD * OR_MAXD * 4];
    mat_transpose(r, n, B, Bt);
    solve_lower_t(n, L, r, Bt, Xt);
    mat_transpose(n, r, Xt, X);
}

/* X = B L^{-T}  (B r x n): solve X L^T = B, i.e. L X^T = B^T */
static void right_solve_lower_t(int r, int n, const double *B, const double *L, double *X)
{
    double Bt[OR_MAXD * OR_MAXD * 4], Xt[OR_MAXD * OR_MAXD * 4];
    mat_transpose(r, n, B, Bt);
    solve_lower(n, L, r, Bt, Xt);
    mat_transpose(n, r, Xt, X);
}

/* Plain Cholesky P = L L^T; returns 0 on success, -1 if not positive definite. */
int or_cholesky(int n, const double *P, double *L)
{
    double tmp[OR_MAXD * OR_MAXD];
    for (int i = 0; i < n * n; ++i)
        tmp[i] = 0.0;
    for (int j = 0; j < n; ++j) {
        double s = P[j * n + j];
        for (int t = 0; t < j; ++t)
            s -= tmp[j * n + t] * tmp[j * n + t];
        if (!(s > 0.0))
            return -1;
        double ljj = sqrt(s);
        tmp[j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double v = P[i * n + j];
            for (int t = 0; t < j; ++t)
                v -= tmp[i * n + t] * tmp[j * n + t];
            tmp[i * n + j] = v / ljj;
        }
    }
    memcpy(L, tmp, sizeof(double) * (size_t)(n * n));
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Tria (Section 2.2): A^T = QR, Tria(A) = R^T, an n x n lower factor with   */
/* Tria(A) Tria(A)^T = A A^T.                                               */
/* Computed here with Givens rotations applied from the right: for each row */
/* i, the entries right of the diagonal are rotated into the diagonal one   */
/* column at a time.  The factor is made unique by a non-negative diagonal. */
/* ------------------------------------------------------------------------ */
void or_tria(int r, int c, const double *A, double *L)
{
    int w = c > r ? c : r; /* zero-pad to at least r columns */
    double W[OR_MAXD * OR_MAXD * 4];
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < w; ++j)
            W[i * w + j] = (j < c) ? A[i * c + j] : 0.0;
    for (int i = 0; i < r; ++i) {
        for (int j = i + 1; j < w; ++j) {
            double a = W[i * w + i], b = W[i * w + j];
            if (b == 0.0)
                continue;
            double rho = hypot(a, b);
            double cs = a / rho, sn = b / rho;
            for (int k = i; k < r; ++k) {
                double x = W[k * w + i], y = W[k * w + j];
                W[k * w + i] = cs * x + sn * y;
                W[k * w + j] = -sn * x + cs * y;
            }
        }
        if (W[i * w + i] < 0.0)
            for (int k = i; k < r; ++k)
                W[k * w + i] = -W[k * w + i];
    }
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < r; ++j)
            L[i * r + j] = (j <= i) ? W[i * w + j] : 0.0;
}

/* DownDate(A, B) (Section 2.2): the lower factor of A A^T - B B^T, obtained */
/* by one rank-1 Cholesky downdate of A per column of B.  A is an n x n      */
/* lower factor, B is n x m.  Returns the number of columns for which the    */
/* downdate broke down (a non-positive radicand); the result then holds NaN. */
int or_downdate(int n, int m, const double *A, const double *B, double *L)
{
    double W[OR_MAXD * OR_MAXD], b[OR_MAXD];
    int bad = 0;
    memcpy(W, A, sizeof(double) * (size_t)(n * n));
    for (int col = 0; col < m; ++col) {
        for (int i = 0; i < n; ++i)
            b[i] = B[i * m + col];
        for (int k = 0; k < n; ++k) {
            double lkk = W[k * n + k];
            double rad = lkk * lkk - b[k] * b[k];
            if (!(rad > 0.0)) {
                if (rad == 0.0 && b[k] == 0.0 && lkk == 0.0)
                    continue; /* zero pivot and nothing to remove */
                bad++;
                rad = NAN;
            }
            double rk = sqrt(rad);
            double cc = rk / lkk, ss = b[k] / lkk;
            W[k * n + k] = rk;
            for (int i = k + 1; i < n; ++i) {
                double lik = (W[i * n + k] - ss * b[i]) / cc;
                b[i] = cc * b[i] - ss * lik;
                W[i * n + k] = lik;
            }
        }
    }
    memcpy(L, W, sizeof(double) * (size_t)(n * n));
    return bad;
}

/* ------------------------------------------------------------------------ */
/* Models (the paper's Section 6.2 coordinated-turn bearings-only model and */
/* a constant-velocity linear model).                                       */
/* prm layout for CT: dt, q1, q2, sigma, s1x, s1y, s2x, s2y                 */
/* ------------------------------------------------------------------------ */

static double sinc_(double u)
{
    if (fabs(u) < 1e-4)
        return 1.0 - u * u / 6.0;
    return sin(u) / u;
}

/* coordinated-turn transition mean E[x_k | x_{k-1}] for x = (px,py,vx,vy,w) */
void or_ct_f(const double *prm, const double *x, double *out)
{
    double dt = prm[0];
    double a = x[4] * dt;
    double s1 = dt * sinc_(a);                           /* sin(w dt)/w        */
    double s2 = dt * 0.5 * a * sinc_(0.5 * a) * sinc_(0.5 * a); /* (1-cos(w dt))/w */
    double ca = cos(a), sa = sin(a);
    double px = x[0], py = x[1], vx = x[2], vy = x[3];
    out[0] = px + s1 * vx - s2 * vy;
    out[1] = py + s2 * vx + s1 * vy;
    out[2] = ca * vx - sa * vy;
    out[3] = sa * vx + ca * vy;
    out[4] = x[4];
}

/* continuous white-noise-acceleration covariance of the CT model */
void or_ct_Q(const double *prm, double *Q)
{
    double dt = prm[0], q1 = prm[1], q2 = prm[2];
    for (int i = 0; i < 25; ++i)
        Q[i] = 0.0;
    Q[0 * 5 + 0] = Q[1 * 5 + 1] = q1 * dt * dt * dt / 3.0;
    Q[0 * 5 + 2] = Q[2 * 5 + 0] = q1 * dt * dt / 2.0;
    Q[1 * 5 + 3] = Q[3 * 5 + 1] = q1 * dt * dt / 2.0;
    Q[2 * 5 + 2] = Q[3 * 5 + 3] = q1 * dt;
    Q[4 * 5 + 4] = q2 * dt;
}

static double wrap_pi(double a)
{ /* to [-pi, pi) */
    const double tp = 2.0 * M_PI;
    double r = fmod(a + M_PI, tp);
    if (r < 0.0)
        r += tp;
    return r - M_PI;
}

/* bearings from the two sensors, each expressed on the branch nearest to  */
/* the reference measurement yref (so the SLR never straddles the cut).     */
void or_ct_h(const double *prm, const double *x, const double *yref, double *out)
{
    double b1 = atan2(x[1] - prm[5], x[0] - prm[4]);
    double b2 = atan2(x[1] - prm[7], x[0] - prm[6]);
    if (yref) {
        out[0] = yref[0] + wrap_pi(b1 - yref[0]);
        out[1] = yref[1] + wrap_pi(b2 - yref[1]);
    } else {
        out[0] = b1;
        out[1] = b2;
    }
}

/* ------------------------------------------------------------------------ */
/* Cubature SLR (Section 4.3).                                             */
/* Sigma points: third-degree spherical-radial rule, 2 nx points            */
/*   X+_i = m + sqrt(nx) N e_i,  X-_i = m - sqrt(nx) N e_i,  weights 1/(2nx)*/
/* Zp, Zm hold the images of X+_i and X-_i as rows (nx rows of nz).         */
/* ------------------------------------------------------------------------ */
void or_sigma_points(int nx, const double *m, const double *N, double *Xp, double *Xm)
{
    double r = sqrt((double)nx);
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < nx; ++j) {
            Xp[i * nx + j] = m[j] + r * N[j * nx + i];
            Xm[i * nx + j] = m[j] - r * N[j * nx + i];
        }
}

/* Residual ("downdate-free") form: with dX the weighted sigma-point        */
/* deviations and Zx the weighted image deviations, the regression matrix   */
/* is G = Zx dX^T (N N^T)^{-1} and Zx Zx^T - G N N^T G^T = R R^T with        */
/* R = Zx - G dX.  For this rule both columns of pair i of R equal          */
/* sqrt(w) ((Z+_i + Z-_i)/2 - zbar), so S = Tria([Snoise, R]) with R scaled  */
/* to nx columns.  Algebraically equal to the Tria + DownDate recipe.       */
int or_slr_residual(int nx, int nz, const double *m, const double *N, const double *Zp,
                    const double *Zm, const double *Snoise, double *G, double *off, double *S)
{
    double zbar[OR_MAXD], D[OR_MAXD * OR_MAXD], R[OR_MAXD * OR_MAXD];
    double w = 1.0 / (2.0 * nx);
    for (int a = 0; a < nz; ++a) {
        double s = 0.0;
        for (int i = 0; i < nx; ++i)
            s += w * (Zp[i * nz + a] + Zm[i * nz + a]);
        zbar[a] = s;
    }
    /* G N = [(Z+_i - Z-_i) / (2 sqrt(nx))]_i  (nz x nx) */
    double h = 1.0 / (2.0 * sqrt((double)nx));
    for (int a = 0; a < nz; ++a)
        for (int i = 0; i < nx; ++i)
            D[a * nx + i] = h * (Zp[i * nz + a] - Zm[i * nz + a]);
    right_solve_lower(nz, nx, D, N, G);
    double Gm[OR_MAXD];
    mat_vec(nz, nx, G, m, Gm);
    for (int a = 0; a < nz; ++a)
        off[a] = zbar[a] - Gm[a];
    double rs = 1.0 / sqrt((double)nx);
    double Aug[OR_MAXD * OR_MAXD * 2];
    for (int a = 0; a < nz; ++a) {
        for (int b = 0; b < nz; ++b)
            Aug[a * (nz + nx) + b] = Snoise[a * nz + b];
        for (int i = 0; i < nx; ++i) {
            R[a * nx + i] = rs * (0.5 * (Zp[i * nz + a] + Zm[i * nz + a]) - zbar[a]);
            Aug[a * (nz + nx) + nz + i] = R[a * nx + i];
        }
    }
    or_tria(nz, nz + nx, Aug, S);
    return 0;
}

/* Literal form of the paper's recipe: zbar; G = sum w (Z - zbar)(X - m)^T */
/* (N N^T)^{-1}; offset zbar - G m; S' = Tria([sqrt(w) Snoise ..., Zx]);    */
/* S = DownDate(S', G N).  Returns the downdate breakdown count.  For an    */
/* additive noise model the weighted noise factors sum to Snoise, so the    */
/* noise block is Snoise itself.                                            */
int or_slr_literal(int nx, int nz, const double *m, const double *N, const double *Zp,
                   const double *Zm, const double *Snoise, double *G, double *off, double *S)
{
    int s = 2 * nx;
    double w = 1.0 / (double)s;
    double Xp[OR_MAXD * OR_MAXD], Xm[OR_MAXD * OR_MAXD];
    or_sigma_points(nx, m, N, Xp, Xm);
    double zbar[OR_MAXD];
    for (int a = 0; a < nz; ++a) {
        double acc = 0.0;
        for (int i = 0; i < nx; ++i)
            acc += w * Zp[i * nz + a] + w * Zm[i * nz + a];
        zbar[a] = acc;
    }
    /* cross-covariance C = sum_i w (Z_i - zbar)(X_i - m)^T  (nz x nx) */
    double C[OR_MAXD * OR_MAXD];
    for (int a = 0; a < nz; ++a)
        for (int b = 0; b < nx; ++b) {
            double acc = 0.0;
            for (int i = 0; i < nx; ++i) {
                acc += w * (Zp[i * nz + a] - zbar[a]) * (Xp[i * nx + b] - m[b]);
                acc += w * (Zm[i * nz + a] - zbar[a]) * (Xm[i * nx + b] - m[b]);
            }
            C[a * nx + b] = acc;
        }
    /* G = C (N N^T)^{-1} = (C N^{-T}) N^{-1} */
    double T1[OR_MAXD * OR_MAXD];
    right_solve_lower_t(nz, nx, C, N, T1);
    right_solve_lower(nz, nx, T1, N, G);
    double Gm[OR_MAXD];
    mat_vec(nz, nx, G, m, Gm);
    for (int a = 0; a < nz; ++a)
        off[a] = zbar[a] - Gm[a];
    /* S' = Tria([Snoise, Zx]) with Zx the weighted deviations (nz x 2nx) */
    int cols = nz + s;
    double Aug[OR_MAXD * OR_MAXD * 4];
    double sw = sqrt(w);
    for (int a = 0; a < nz; ++a) {
        for (int b = 0; b < nz; ++b)
            Aug[a * cols + b] = Snoise[a * nz + b];
        for (int i = 0; i < nx; ++i) {
            Aug[a * cols + nz + i] = sw * (Zp[i * nz + a] - zbar[a]);
            Aug[a * cols + nz + nx + i] = sw * (Zm[i * nz + a] - zbar[a]);
        }
    }
    double Sp[OR_MAXD * OR_MAXD];
    or_tria(nz, cols, Aug, Sp);
    double GN[OR_MAXD * OR_MAXD];
    mat_mul(nz, nx, nx, G, N, GN);
    return or_downdate(nz, nx, Sp, GN, S);
}

/* ------------------------------------------------------------------------ */
/* Sequential square-root Kalman filter (the algebra of Tables 1-2 applied */
/* as a recursion; Algorithm 1 computes the same marginals by a scan).      */
/* ell[j] = log N(y_{j+1}; predicted mean, predicted covariance): the full  */
/* Gaussian log density including the -(ny/2) log(2 pi) constant.           */
/* ------------------------------------------------------------------------ */
/* Sigma-point rules with positive weights (Section 4.3).  A rule is a set  */
/* of unit points xi_i (nx each) with weights w_i > 0 summing to one that    */
/* integrates the first and second moments of N(0, I) exactly; for the      */
/* Gaussian N(m, N N^T) its points are X_i = m + N xi_i.  The cubature,      */
/* unscented and Gauss-Hermite rules are built by the Python wrapper and     */
/* installed here with or_set_rule; linearisation method OR_RULE reads it.  */
/* (The rule table is process-global: one rule at a time.)                  */
/* ------------------------------------------------------------------------ */
#define OR_RULE 3
#define OR_MAXPTS 4096
static int g_rule_nx = 0, g_rule_np = 0;
static double g_rule_xi[OR_MAXPTS * 8], g_rule_w[OR_MAXPTS];

int or_set_rule(int nx, int np, const double *xi, const double *w)
{
    if (nx < 1 || nx > 8 || np < 1 || np > OR_MAXPTS)
        return -1;
    g_rule_nx = nx;
    g_rule_np = np;
    memcpy(g_rule_xi, xi, sizeof(double) * (size_t)(np * nx));
    memcpy(g_rule_w, w, sizeof(double) * (size_t)np);
    return 0;
}

/* X_i = m + N xi_i for the installed rule ([np][nx]) */
static void rule_points(int nx, const double *m, const double *N, double *X)
{
    for (int i = 0; i < g_rule_np; ++i)
        for (int a = 0; a < nx; ++a) {
            double s = m[a];
            for (int b = 0; b <= a; ++b)
                s += N[a * nx + b] * g_rule_xi[i * nx + b];
            X[i * nx + a] = s;
        }
}

/* L <- Tria([L, B]) for an nz x nz lower L and an nz x m block B, taking   */
/* the columns of B a few at a time (Tria([A, B]) = Tria([Tria(A), B])).    */
static void tria_accumulate(int nz, double *L, int m, const double *B)
{
    enum { CH = 16 };
    double A[OR_MAXD * (OR_MAXD + CH)];
    for (int c0 = 0; c0 < m; c0 += CH) {
        int mc = m - c0 < CH ? m - c0 : CH;
        int w = nz + mc;
        for (int a = 0; a < nz; ++a) {
            for (int b = 0; b < nz; ++b)
                A[a * w + b] = L[a * nz + b];
            for (int q = 0; q < mc; ++q)
                A[a * w + nz + q] = B[(long)a * m + c0 + q];
        }
        or_tria(nz, w, A, L);
    }
}

/* Generalised statistical linear regression (the GSLR moments of Section   */
/* 2.3 with the sigma-point approximations of Section 4.3) of a conditional */
/* model with mean g(x) and lower covariance factor Sg(x), at N(m, N N^T):  */
/*   Z_i = g(X_i),  zbar = sum_i w_i Z_i,                                   */
/*   G   = [sum_i w_i (Z_i - zbar)(X_i - m)^T] (N N^T)^{-1},                */
/*   off = zbar - G m,                                                      */
/*   S S^T = sum_i w_i Sg(X_i) Sg(X_i)^T + Zx Zx^T - G N N^T G^T,            */
/*   Zx = [sqrt(w_i)(Z_i - zbar)]_i.                                        */
/* The first sum is E[V[y|x]]; with additive noise it is Snoise Snoise^T    */
/* (pass Snoise, Sg = NULL), else pass the per-point factors Sg [np][nz][nz].*/
/* literal = 0: S = Tria([noise columns, sqrt(w_i)(Z_i - zbar - G(X_i - m))]),*/
/*   whose residual columns have Gram matrix Zx Zx^T - G N N^T G^T exactly   */
/*   because the rule integrates second moments exactly;                    */
/* literal = 1: the printed S = DownDate(Tria([noise columns, Zx]), G N).    */
/* Returns the downdate breakdown count (0 for literal = 0).                */
int or_slr_rule(int nx, int nz, int np, const double *X, const double *w, const double *m,
                const double *N, const double *Z, const double *Sg, const double *Snoise,
                int literal, double *G, double *off, double *S)
{
    double zbar[OR_MAXD], C[OR_MAXD * OR_MAXD], T1[OR_MAXD * OR_MAXD], Gm[OR_MAXD];
    for (int a = 0; a < nz; ++a) {
        double s = 0.0;
        for (int i = 0; i < np; ++i)
            s += w[i] * Z[i * nz + a];
        zbar[a] = s;
    }
    for (int a = 0; a < nz; ++a)
        for (int b = 0; b < nx; ++b) {
            double s = 0.0;
            for (int i = 0; i < np; ++i)
                s += w[i] * (Z[i * nz + a] - zbar[a]) * (X[i * nx + b] - m[b]);
            C[a * nx + b] = s;
        }
    /* (N N^T)^{-1} = N^{-T} N^{-1} */
    right_solve_lower_t(nz, nx, C, N, T1);
    right_solve_lower(nz, nx, T1, N, G);
    mat_vec(nz, nx, G, m, Gm);
    for (int a = 0; a < nz; ++a)
        off[a] = zbar[a] - Gm[a];
    /* noise part */
    double L[OR_MAXD * OR_MAXD];
    for (int q = 0; q < nz * nz; ++q)
        L[q] = 0.0;
    if (Snoise) {
        for (int a = 0; a < nz; ++a)
            for (int b = 0; b < nz; ++b)
                L[a * nz + b] = (b <= a) ? Snoise[a * nz + b] : 0.0;
    } else {
        int mc = np * nz;
        double *B = malloc(sizeof(double) * (size_t)nz * (size_t)mc);
        for (int i = 0; i < np; ++i) {
            double sw = sqrt(w[i]);
            for (int a = 0; a < nz; ++a)
                for (int b = 0; b < nz; ++b)
                    B[(long)a * mc + i * nz + b] = sw * Sg[(long)i * nz * nz + a * nz + b];
        }
        tria_accumulate(nz, L, mc, B);
        free(B);
    }
    double *R = malloc(sizeof(double) * (size_t)nz * (size_t)np);
    for (int i = 0; i < np; ++i) {
        double sw = sqrt(w[i]), dx[OR_MAXD], gd[OR_MAXD];
        for (int b = 0; b < nx; ++b)
            dx[b] = X[i * nx + b] - m[b];
        mat_vec(nz, nx, G, dx, gd);
        for (int a = 0; a < nz; ++a)
            R[(long)a * np + i] = sw * (Z[i * nz + a] - zbar[a] - (literal ? 0.0 : gd[a]));
    }
    tria_accumulate(nz, L, np, R);
    free(R);
    int bad = 0;
    if (literal) {
        double GN[OR_MAXD * OR_MAXD];
        mat_mul(nz, nx, nx, G, N, GN);
        bad = or_downdate(nz, nx, L, GN, S);
    } else {
        memcpy(S, L, sizeof(double) * (size_t)(nz * nz));
    }
    return bad;
}

/* ------------------------------------------------------------------------ */
int or_sqrt_filter(int n, int nx, int ny, const double *m0, const double *N0, const double *F,
                   const double *c, const double *SL, const double *H, const double *d,
                   const double *SO, long gstride, const double *y, double *mf, double *Nf,
                   double *ell)
{
    memcpy(mf, m0, sizeof(double) * (size_t)nx);
    memcpy(Nf, N0, sizeof(double) * (size_t)(nx * nx));
    for (int j = 0; j < n; ++j) {
        long g = gstride * j;
        const double *Fj = F + g * nx * nx, *cj = c + g * nx, *SLj = SL + g * nx * nx;
        const double *Hj = H + g * ny * nx, *dj = d + g * ny, *SOj = SO + g * ny * ny;
        const double *m = mf + (long)j * nx, *Nm = Nf + (long)j * nx * nx;
        double mp[OR_MAXD], Np[OR_MAXD * OR_MAXD], FN[OR_MAXD * OR_MAXD];
        double Aug[OR_MAXD * OR_MAXD * 4];
        /* predicted mean and square-root covariance */
        mat_vec(nx, nx, Fj, m, mp);
        for (int i = 0; i < nx; ++i)
            mp[i] += cj[i];
        mat_mul(nx, nx, nx, Fj, Nm, FN);
        for (int i = 0; i < nx; ++i)
            for (int t = 0; t < nx; ++t) {
                Aug[i * 2 * nx + t] = FN[i * nx + t];
                Aug[i * 2 * nx + nx + t] = SLj[i * nx + t];
            }
        or_tria(nx, 2 * nx, Aug, Np);
        /* Psi = Tria([[H N-, S_Omega], [N-, 0]]) */
        int R = ny + nx, Cc = nx + ny;
        double HN[OR_MAXD * OR_MAXD], Psi[OR_MAXD * OR_MAXD * 4];
        mat_mul(ny, nx, nx, Hj, Np, HN);
        for (int i = 0; i < R * Cc; ++i)
            Aug[i] = 0.0;
        for (int i = 0; i < ny; ++i) {
            for (int t = 0; t < nx; ++t)
                Aug[i * Cc + t] = HN[i * nx + t];
            for (int t = 0; t < ny; ++t)
                Aug[i * Cc + nx + t] = SOj[i * ny + t];
        }
        for (int i = 0; i < nx; ++i)
            for (int t = 0; t < nx; ++t)
                Aug[(ny + i) * Cc + t] = Np[i * nx + t];
        or_tria(R, Cc, Aug, Psi);
        double P11[OR_MAXD * OR_MAXD], P21[OR_MAXD * OR_MAXD];
        for (int i = 0; i < ny; ++i)
            for (int t = 0; t < ny; ++t)
                P11[i * ny + t] = Psi[i * R + t];
        for (int i = 0; i < nx; ++i)
            for (int t = 0; t < ny; ++t)
                P21[i * ny + t] = Psi[(ny + i) * R + t];
        /* innovation */
        double v[OR_MAXD], Hm[OR_MAXD], u[OR_MAXD];
        mat_vec(ny, nx, Hj, mp, Hm);
        for (int i = 0; i < ny; ++i)
            v[i] = y[(long)j * ny + i] - Hm[i] - dj[i];
        solve_lower(ny, P11, 1, v, u); /* u = Psi11^{-1} v */
        double* mo = mf + (long)(j + 1) * nx;
        double* No = Nf + (long)(j + 1) * nx * nx;
        double Ku[OR_MAXD];
        mat_vec(nx, ny, P21, u, Ku);
        for (int i = 0; i < nx; ++i)
            mo[i] = mp[i] + Ku[i];
        for (int i = 0; i < nx; ++i)
            for (int t = 0; t < nx; ++t)
                No[i * nx + t] = Psi[(ny + i) * R + ny + t];
        if (ell) {
            double l = -0.5 * ny * log(2.0 * M_PI);
            for (int i = 0; i < ny; ++i)
                l -= log(fabs(P11[i * ny + i]));
            for (int i = 0; i < ny; ++i)
                l -= 0.5 * u[i] * u[i];
            ell[j] = l;
        }
    }
    return 0;
}

/* Sequential square-root RTS smoother (Table 4 algebra as a recursion).    */
/* Optional Eout[k] receives the smoother gain E_k (k = 0..n-1).           */
int or_sqrt_smoother(int n, int nx, const double *F, const double *c, const double *SL,
                     long gstride, const double *mf, const double *Nf, double *ms, double *Ns,
                     double *Eout)
{
    memcpy(ms + (long)n * nx, mf + (long)n * nx, sizeof(double) * (size_t)nx);
    memcpy(Ns + (long)n * nx * nx, Nf + (long)n * nx * nx, sizeof(double) * (size_t)(nx * nx));
    for (int k = n - 1; k >= 0; --k) {
        long g = gstride * k;
        const double *Fk = F + g * nx * nx, *ck = c + g * nx, *SLk = SL + g * nx * nx;
        const double *m = mf + (long)k * nx, *Nm = Nf + (long)k * nx * nx;
        int R = 2 * nx;
        double Aug[OR_MAXD * OR_MAXD * 4], Phi[OR_MAXD * OR_MAXD * 4], FN[OR_MAXD * OR_MAXD];
        mat_mul(nx, nx, nx, Fk, Nm, FN);
        for (int i = 0; i < R * R; ++i)
            Aug[i] = 0.0;
        for (int i = 0; i < nx; ++i)
            for (int t = 0; t < nx; ++t) {
                Aug[i * R + t] = FN[i * nx + t];
                Aug[i * R + nx + t] = SLk[i * nx + t];
                Aug[(nx + i) * R + t] = Nm[i * nx + t];
            }
        or_tria(R, R, Aug, Phi);
        double P11[OR_MAXD * OR_MAXD], P21[OR_MAXD * OR_MAXD], P22[OR_MAXD * OR_MAXD];
        for (int i = 0; i < nx; ++i)
            for (int t = 0; t < nx; ++t) {
                P11[i * nx + t] = Phi[i * R + t];
                P21[i * nx + t] = Phi[(nx + i) * R + t];
                P22[i * nx + t] = Phi[(nx + i) * R + nx + t];
            }
        double E[OR_MAXD * OR_MAXD];
        right_solve_lower(nx, nx, P21, P11, E); /* E = Phi21 Phi11^{-1} */
        double Fm[OR_MAXD], r[OR_MAXD], Er[OR_MAXD];
        mat_vec(nx, nx, Fk, m, Fm);
        for (int i = 0; i < nx; ++i)
            r[i] = ms[(long)(k + 1) * nx + i] - Fm[i] - ck[i];
        mat_vec(nx, nx, E, r, Er);
        for (int i = 0; i < nx; ++i)
            ms[(long)k * nx + i] = m[i] + Er[i];
        double EN[OR_MAXD * OR_MAXD];
        mat_mul(nx, nx, nx, E, Ns + (long)(k + 1) * nx * nx, EN);
        for (int i = 0; i < nx; ++i)
            for (int t = 0; t < nx; ++t) {
                Aug[i * 2 * nx + t] = EN[i * nx + t];
                Aug[i * 2 * nx + nx + t] = P22[i * nx + t];
            }
        or_tria(nx, 2 * nx, Aug, Ns + (long)k * nx * nx);
        if (Eout)
            memcpy(Eout + (long)k * nx * nx, E, sizeof(double) * (size_t)(nx * nx));
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Covariance-form Kalman filter and RTS smoother (textbook; cross-check).  */
/* Covariances Lam = S_Lambda S_Lambda^T and Om = S_Omega S_Omega^T.        */
/* ------------------------------------------------------------------------ */
int or_cov_filter(int n, int nx, int ny, const double *m0, const double *P0, const double *F,
                  const double *c, const double *Lam, const double *H, const double *d,
                  const double *Om, long gstride, const double *y, double *mf, double *Pf,
                  double *mp_out, double *Pp_out, double *ell)
{
    memcpy(mf, m0, sizeof(double) * (size_t)nx);
    memcpy(Pf, P0, sizeof(double) * (size_t)(nx * nx));
    for (int j = 0; j < n; ++j) {
        long g = gstride * j;
        const double *Fj = F + g * nx * nx, *cj = c + g * nx, *Lj = Lam + g * nx * nx;
        const double *Hj = H + g * ny * nx, *dj = d + g * ny, *Oj = Om + g * ny * ny;
        double mp[OR_MAXD], Pp[OR_MAXD * OR_MAXD], T[OR_MAXD * OR_MAXD];
        mat_vec(nx, nx, Fj, mf + (long)j * nx, mp);
        for (int i = 0; i < nx; ++i)
            mp[i] += cj[i];
        mat_mul(nx, nx, nx, Fj, Pf + (long)j * nx * nx, T);
        mat_mult(nx, nx, nx, T, Fj, Pp);
        for (int i = 0; i < nx * nx; ++i)
            Pp[i] += Lj[i];
        if (mp_out)
            memcpy(mp_out + (long)j * nx, mp, sizeof(double) * (size_t)nx);
        if (Pp_out)
            memcpy(Pp_out + (long)j * nx * nx, Pp, sizeof(double) * (size_t)(nx * nx));
        double HP[OR_MAXD * OR_MAXD], S[OR_MAXD * OR_MAXD], LS[OR_MAXD * OR_MAXD];
        mat_mul(ny, nx, nx, Hj, Pp, HP);
        mat_mult(ny, nx, ny, HP, Hj, S);
        for (int i = 0; i < ny * ny; ++i)
            S[i] += Oj[i];
        if (or_cholesky(ny, S, LS) != 0)
            return -1;
        double v[OR_MAXD], Hm[OR_MAXD];
        mat_vec(ny, nx, Hj, mp, Hm);
        for (int i = 0; i < ny; ++i)
            v[i] = y[(long)j * ny + i] - Hm[i] - dj[i];
        /* K = P- H^T S^{-1} ; K^T = S^{-1} H P- */
        double Kt[OR_MAXD * OR_MAXD], tmp[OR_MAXD * OR_MAXD];
        solve_lower(ny, LS, nx, HP, tmp);
        solve_lower_t(ny, LS, nx, tmp, Kt);
        double Sv[OR_MAXD], Sv2[OR_MAXD];
        solve_lower(ny, LS, 1, v, Sv);
        solve_lower_t(ny, LS, 1, Sv, Sv2);
        double *mo = mf + (long)(j + 1) * nx, *Po = Pf + (long)(j + 1) * nx * nx;
        for (int i = 0; i < nx; ++i) {
            double s = mp[i];
            for (int a = 0; a < ny; ++a)
                s += Kt[a * nx + i] * v[a];
            mo[i] = s;
        }
        /* P = P- - K S K^T = P- - (H P-)^T S^{-1} (H P-) */
        for (int i = 0; i < nx; ++i)
            for (int t = 0; t < nx; ++t) {
                double s = Pp[i * nx + t];
                for (int a = 0; a < ny; ++a)
                    s -= HP[a * nx + i] * Kt[a * nx + t];
                Po[i * nx + t] = s;
            }
        for (int i = 0; i < nx; ++i) /* symmetrise */
            for (int t = 0; t < i; ++t) {
                double s = 0.5 * (Po[i * nx + t] + Po[t * nx + i]);
                Po[i * nx + t] = Po[t * nx + i] = s;
            }
        if (ell) {
            double l = -0.5 * ny * log(2.0 * M_PI);
            for (int i = 0; i < ny; ++i)
                l -= log(LS[i * ny + i]);
            for (int i = 0; i < ny; ++i)
                l -= 0.5 * Sv[i] * Sv[i];
            ell[j] = l;
        }
    }
    return 0;
}

int or_cov_smoother(int n, int nx, const double *F, const double *c, const double *Lam,
                    long gstride, const double *mf, const double *Pf, double *ms, double *Ps,
                    double *Gout)
{
    memcpy(ms + (long)n * nx, mf + (long)n * nx, sizeof(double) * (size_t)nx);
    memcpy(Ps + (long)n * nx * nx, Pf + (long)n * nx * nx, sizeof(double) * (size_t)(nx * nx));
    for (int k = n - 1; k >= 0; --k) {
        long g = gstride * k;
        const double *Fk = F + g * nx * nx, *ck = c + g * nx, *Lk = Lam + g * nx * nx;
        const double *m = mf + (long)k * nx, *P = Pf + (long)k * nx * nx;
        double mp[OR_MAXD], Pp[OR_MAXD * OR_MAXD], T[OR_MAXD * OR_MAXD], L[OR_MAXD * OR_MAXD];
        mat_vec(nx, nx, Fk, m, mp);
        for (int i = 0; i < nx; ++i)
            mp[i] += ck[i];
        mat_mul(nx, nx, nx, Fk, P, T); /* T = F P */
        mat_mult(nx, nx, nx, T, Fk, Pp);
        for (int i = 0; i < nx * nx; ++i)
            Pp[i] += Lk[i];
        if (or_cholesky(nx, Pp, L) != 0)
            return -1;
        /* G = P F^T Pp^{-1}; G^T = Pp^{-1} F P = Pp^{-1} T */
        double tmp[OR_MAXD * OR_MAXD], Gt[OR_MAXD * OR_MAXD], G[OR_MAXD * OR_MAXD];
        solve_lower(nx, L, nx, T, tmp);
        solve_lower_t(nx, L, nx, tmp, Gt);
        mat_transpose(nx, nx, Gt, G);
        double dm[OR_MAXD], Gdm[OR_MAXD];
        for (int i = 0; i < nx; ++i)
            dm[i] = ms[(long)(k + 1) * nx + i] - mp[i];
        mat_vec(nx, nx, G, dm, Gdm);
        for (int i = 0; i < nx; ++i)
            ms[(long)k * nx + i] = m[i] + Gdm[i];
        double dP[OR_MAXD * OR_MAXD], GdP[OR_MAXD * OR_MAXD], Po[OR_MAXD * OR_MAXD];
        for (int i = 0; i < nx * nx; ++i)
            dP[i] = Ps[(long)(k + 1) * nx * nx + i] - Pp[i];
        mat_mul(nx, nx, nx, G, dP, GdP);
        mat_mult(nx, nx, nx, GdP, G, Po);
        for (int i = 0; i < nx * nx; ++i)
            Po[i] += P[i];
        for (int i = 0; i < nx; ++i)
            for (int t = 0; t < i; ++t) {
                double s = 0.5 * (Po[i * nx + t] + Po[t * nx + i]);
                Po[i * nx + t] = Po[t * nx + i] = s;
            }
        memcpy(Ps + (long)k * nx * nx, Po, sizeof(double) * (size_t)(nx * nx));
        if (Gout)
            memcpy(Gout + (long)k * nx * nx, G, sizeof(double) * (size_t)(nx * nx));
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Parallel-form elements and combination operators (Lemmas 1-4).          */
/* Filter element: A (nx x nx), b (nx), U (nx x nx), eta (nx), Z (nx x nx). */
/* Smoother element: E (nx x nx), g (nx), D (nx x nx).                      */
/* ------------------------------------------------------------------------ */

/* Z_k is nx x ny; Lemma 1's proof squares it by zero columns when nx > ny */
/* and replaces it by Tria(Z) when nx < ny.                                 */
static void square_Z(int nx, int ny, const double *Zr, double *Z)
{
    if (nx >= ny) {
        for (int i = 0; i < nx; ++i)
            for (int t = 0; t < nx; ++t)
                Z[i * nx + t] = (t < ny) ? Zr[i * ny + t] : 0.0;
    } else {
        or_tria(nx, ny, Zr, Z);
    }
}

/* Table 1 (k = 1), square-root column. */
void or_filter_element_first(int nx, int ny, const double *m0, const double *N0, const double *F0,
                             const double *c0, const double *SL0, const double *H1,
                             const double *d1, const double *SO1, const double *y1, double *A,
                             double *b, double *U, double *eta, double *Z)
{
    double mp[OR_MAXD], Np[OR_MAXD * OR_MAXD], FN[OR_MAXD * OR_MAXD], Aug[OR_MAXD * OR_MAXD * 4];
    mat_vec(nx, nx, F0, m0, mp);
    for (int i = 0; i < nx; ++i)
        mp[i] += c0[i];
    mat_mul(nx, nx, nx, F0, N0, FN);
    for (int i = 0; i < nx; ++i)
        for (int t = 0; t < nx; ++t) {
            Aug[i * 2 * nx + t] = FN[i * nx + t];
            Aug[i * 2 * nx + nx + t] = SL0[i * nx + t];
        }
    or_tria(nx, 2 * nx, Aug, Np);
    int R = ny + nx, C = nx + ny;
    double HN[OR_MAXD * OR_MAXD], Psi[OR_MAXD * OR_MAXD * 4];
    mat_mul(ny, nx, nx, H1, Np, HN);
    for (int i = 0; i < R * C; ++i)
        Aug[i] = 0.0;
    for (int i = 0; i < ny; ++i) {
        for (int t = 0; t < nx; ++t)
            Aug[i * C + t] = HN[i * nx + t];
        for (int t = 0; t < ny; ++t)
            Aug[i * C + nx + t] = SO1[i * ny + t];
    }
    for (int i = 0; i < nx; ++i)
        for (int t = 0; t < nx; ++t)
            Aug[(ny + i) * C + t] = Np[i * nx + t];
    or_tria(R, C, Aug, Psi);
    double Y[OR_MAXD * OR_MAXD], P21[OR_MAXD * OR_MAXD], K[OR_MAXD * OR_MAXD];
    for (int i = 0; i < ny; ++i)
        for (int t = 0; t < ny; ++t)
            Y[i * ny + t] = Psi[i * R + t];
    for (int i = 0; i < nx; ++i)
        for (int t = 0; t < ny; ++t)
            P21[i * ny + t] = Psi[(ny + i) * R + t];
    right_solve_lower(nx, ny, P21, Y, K); /* K1 = Psi21 Psi11^{-1} */
    for (int i = 0; i < nx * nx; ++i)
        A[i] = 0.0;
    double v[OR_MAXD], Hm[OR_MAXD], Kv[OR_MAXD];
    mat_vec(ny, nx, H1, mp, Hm);
    for (int i = 0; i < ny; ++i)
        v[i] = y1[i] - Hm[i] - d1[i];
    mat_vec(nx, ny, K, v, Kv);
    for (int i = 0; i < nx; ++i)
        b[i] = mp[i] + Kv[i];
    for (int i = 0; i < nx; ++i)
        for (int t = 0; t < nx; ++t)
            U[i * nx + t] = Psi[(ny + i) * R + ny + t];
    /* Z1 = F0^T H1^T Y1^{-T} (nx x ny) */
    double HF[OR_MAXD * OR_MAXD], HFt[OR_MAXD * OR_MAXD], Zr[OR_MAXD * OR_MAXD];
    mat_mul(ny, nx, nx, H1, F0, HF);
    mat_transpose(ny, nx, HF, HFt);
    right_solve_lower_t(nx, ny, HFt, Y, Zr);
    /* eta1 = Z1 Y1^{-1} (y1 - H1 c0 - d1) */
    double r[OR_MAXD], Hc[OR_MAXD], Yr[OR_MAXD];
    mat_vec(ny, nx, H1, c0, Hc);
    for (int i = 0; i < ny; ++i)
        r[i] = y1[i] - Hc[i] - d1[i];
    solve_lower(ny, Y, 1, r, Yr);
    mat_vec(nx, ny, Zr, Yr, eta);
    square_Z(nx, ny, Zr, Z);
}

/* Table 2 (1 < k <= n), square-root column.  b_k uses d_k (the measurement */
/* offset of the same step, as in eta_k and the model).                     */
void or_filter_element(int nx, int ny, const double *Fk1, const double *ck1, const double *SLk1,
                       const double *Hk, const double *dk, const double *SOk, const double *yk,
                       double *A, double *b, double *U, double *eta, double *Z)
{
    int R = ny + nx, C = nx + ny;
    double HS[OR_MAXD * OR_MAXD], Aug[OR_MAXD * OR_MAXD * 4], Psi[OR_MAXD * OR_MAXD * 4];
    mat_mul(ny, nx, nx, Hk, SLk1, HS);
    for (int i = 0; i < R * C; ++i)
        Aug[i] = 0.0;
    for (int i = 0; i < ny; ++i) {
        for (int t = 0; t < nx; ++t)
            Aug[i * C + t] = HS[i * nx + t];
        for (int t = 0; t < ny; ++t)
            Aug[i * C + nx + t] = SOk[i * ny + t];
    }
    for (int i = 0; i < nx; ++i)
        for (int t = 0; t < nx; ++t)
            Aug[(ny + i) * C + t] = SLk1[i * nx + t];
    or_tria(R, C, Aug, Psi);
    double Y[OR_MAXD * OR_MAXD], P21[OR_MAXD * OR_MAXD], K[OR_MAXD * OR_MAXD];
    for (int i = 0; i < ny; ++i)
        for (int t = 0; t < ny; ++t)
            Y[i * ny + t] = Psi[i * R + t];
    for (int i = 0; i < nx; ++i)
        for (int t = 0; t < ny; ++t)
            P21[i * ny + t] = Psi[(ny + i) * R + t];
    right_solve_lower(nx, ny, P21, Y, K);
    /* A = (I - K H) F */
    double KH[OR_MAXD * OR_MAXD], IKH[OR_MAXD * OR_MAXD];
    mat_mul(nx, ny, nx, K, Hk, KH);
    eye(nx, IKH);
    for (int i = 0; i < nx * nx; ++i)
        IKH[i] -= KH[i];
    mat_mul(nx, nx, nx, IKH, Fk1, A);
    double r[OR_MAXD], Hc[OR_MAXD], Kr[OR_MAXD];
    mat_vec(ny, nx, Hk, ck1, Hc);
    for (int i = 0; i < ny; ++i)
        r[i] = yk[i] - Hc[i] - dk[i];
    mat_vec(nx, ny, K, r, Kr);
    for (int i = 0; i < nx; ++i)
        b[i] = ck1[i] + Kr[i];
    for (int i = 0; i < nx; ++i)
        for (int t = 0; t < nx; ++t)
            U[i * nx + t] = Psi[(ny + i) * R + ny + t];
    double HF[OR_MAXD * OR_MAXD], HFt[OR_MAXD * OR_MAXD], Zr[OR_MAXD * OR_MAXD], Yr[OR_MAXD];
    mat_mul(ny, nx, nx, Hk, Fk1, HF);
    mat_transpose(ny, nx, HF, HFt);
    right_solve_lower_t(nx, ny, HFt, Y, Zr);
    solve_lower(ny, Y, 1, r, Yr);
    mat_vec(nx, ny, Zr, Yr, eta);
    square_Z(nx, ny, Zr, Z);
}

/* Table 3, square-root column: (i) (x) (j). Outputs may alias nothing.     */
void or_filter_combine(int nx, const double *Ai, const double *bi, const double *Ui,
                       const double *etai, const double *Zi, const double *Aj, const double *bj,
                       const double *Uj, const double *etaj, const double *Zj, double *A,
                       double *b, double *U, double *eta, double *Z)
{
    int R = 2 * nx;
    double UtZ[OR_MAXD * OR_MAXD], Aug[OR_MAXD * OR_MAXD * 4], Xi[OR_MAXD * OR_MAXD * 4];
    mat_tmul(nx, nx, nx, Ui, Zj, UtZ);
    for (int i = 0; i < R * R; ++i)
        Aug[i] = 0.0;
    for (int i = 0; i < nx; ++i) {
        for (int t = 0; t < nx; ++t) {
            Aug[i * R + t] = UtZ[i * nx + t];
            Aug[(nx + i) * R + t] = Zj[i * nx + t];
        }
        Aug[i * R + nx + i] = 1.0;
    }
    or_tria(R, R, Aug, Xi);
    double X11[OR_MAXD * OR_MAXD], X21[OR_MAXD * OR_MAXD], X22[OR_MAXD * OR_MAXD];
    for (int i = 0; i < nx; ++i)
        for (int t = 0; t < nx; ++t) {
            X11[i * nx + t] = Xi[i * R + t];
            X21[i * nx + t] = Xi[(nx + i) * R + t];
            X22[i * nx + t] = Xi[(nx + i) * R + nx + t];
        }
    /* W = U_i Xi11^{-T} ; Mt = I - W Xi21^T  (= (I + C_i J_j)^{-1}) */
    double W[OR_MAXD * OR_MAXD], WX[OR_MAXD * OR_MAXD], Mt[OR_MAXD * OR_MAXD];
    right_solve_lower_t(nx, nx, Ui, X11, W);
    mat_mult(nx, nx, nx, W, X21, WX);
    eye(nx, Mt);
    for (int i = 0; i < nx * nx; ++i)
        Mt[i] -= WX[i];
    double AjM[OR_MAXD * OR_MAXD];
    mat_mul(nx, nx, nx, Aj, Mt, AjM);
    mat_mul(nx, nx, nx, AjM, Ai, A); /* A_ij = A_j A_i - A_j U_i Xi11^{-T} Xi21^T A_i */
    double UtEta[OR_MAXD], UUeta[OR_MAXD], tmp[OR_MAXD], tb[OR_MAXD];
    mat_tvec(nx, nx, Ui, etaj, UtEta);
    mat_vec(nx, nx, Ui, UtEta, UUeta);
    for (int i = 0; i < nx; ++i)
        tmp[i] = bi[i] + UUeta[i];
    mat_vec(nx, nx, AjM, tmp, tb);
    for (int i = 0; i < nx; ++i)
        b[i] = tb[i] + bj[i];
    double AjW[OR_MAXD * OR_MAXD];
    mat_mul(nx, nx, nx, Aj, W, AjW);
    for (int i = 0; i < nx; ++i)
        for (int t = 0; t < nx; ++t) {
            Aug[i * 2 * nx + t] = AjW[i * nx + t];
            Aug[i * 2 * nx + nx + t] = Uj[i * nx + t];
        }
    or_tria(nx, 2 * nx, Aug, U);
    /* eta_ij = A_i^T (I - Xi21 Xi11^{-1} U_i^T)(eta_j - Z_j Z_j^T b_i) + eta_i;  */
    /* the bracket is Mt^T                                                       */
    double Ztb[OR_MAXD], ZZb[OR_MAXD], r[OR_MAXD], Mr[OR_MAXD], Ar[OR_MAXD];
    mat_tvec(nx, nx, Zj, bi, Ztb);
    mat_vec(nx, nx, Zj, Ztb, ZZb);
    for (int i = 0; i < nx; ++i)
        r[i] = etaj[i] - ZZb[i];
    mat_tvec(nx, nx, Mt, r, Mr);
    mat_tvec(nx, nx, Ai, Mr, Ar);
    for (int i = 0; i < nx; ++i)
        eta[i] = Ar[i] + etai[i];
    double AtX[OR_MAXD * OR_MAXD];
    mat_tmul(nx, nx, nx, Ai, X22, AtX);
    for (int i = 0; i < nx; ++i)
        for (int t = 0; t < nx; ++t) {
            Aug[i * 2 * nx + t] = AtX[i * nx + t];
            Aug[i * 2 * nx + nx + t] = Zi[i * nx + t];
        }
    or_tria(nx, 2 * nx, Aug, Z);
}

/* Table 4, square-root column, for 0 <= k < n (the caller sets the last    */
/* element to E = 0, g = m^f_n, D = N^f_n).                                 */
void or_smoother_element(int nx, const double *Fk, const double *ck, const double *SLk,
                         const double *mf, const double *Nf, double *E, double *g, double *D)
{
    int R = 2 * nx;
    double FN[OR_MAXD * OR_MAXD], Aug[OR_MAXD * OR_MAXD * 4], Phi[OR_MAXD * OR_MAXD * 4];
    mat_mul(nx, nx, nx, Fk, Nf, FN);
    for (int i = 0; i < R * R; ++i)
        Aug[i] = 0.0;
    for (int i = 0; i < nx; ++i)
        for (int t = 0; t < nx; ++t) {
            Aug[i * R + t] = FN[i * nx + t];
            Aug[i * R + nx + t] = SLk[i * nx + t];
            Aug[(nx + i) * R + t] = Nf[i * nx + t];
        }
    or_tria(R, R, Aug, Phi);
    double P11[OR_MAXD * OR_MAXD], P21[OR_MAXD * OR_MAXD];
    for (int i = 0; i < nx; ++i)
        for (int t = 0; t < nx; ++t) {
            P11[i * nx + t] = Phi[i * R + t];
            P21[i * nx + t] = Phi[(nx + i) * R + t];
            D[i * nx + t] = Phi[(nx + i) * R + nx + t];
        }
    right_solve_lower(nx, nx, P21, P11, E);
    double Fm[OR_MAXD], Eg[OR_MAXD];
    mat_vec(nx, nx, Fk, mf, Fm);
    for (int i = 0; i < nx; ++i)
        Fm[i] += ck[i];
    mat_vec(nx, nx, E, Fm, Eg);
    for (int i = 0; i < nx; ++i)
        g[i] = mf[i] - Eg[i];
}

/* Table 5, square-root column: (i) (x) (j). */
void or_smoother_combine(int nx, const double *Ei, const double *gi, const double *Di,
                         const double *Ej, const double *gj, const double *Dj, double *E,
                         double *g, double *D)
{
    double EE[OR_MAXD * OR_MAXD], Eg[OR_MAXD], ED[OR_MAXD * OR_MAXD], Aug[OR_MAXD * OR_MAXD * 2];
    mat_mul(nx, nx, nx, Ei, Ej, EE);
    mat_vec(nx, nx, Ei, gj, Eg);
    mat_mul(nx, nx, nx, Ei, Dj, ED);
    for (int i = 0; i < nx; ++i)
        for (int t = 0; t < nx; ++t) {
            Aug[i * 2 * nx + t] = ED[i * nx + t];
            Aug[i * 2 * nx + nx + t] = Di[i * nx + t];
        }
    double Dn[OR_MAXD * OR_MAXD];
    or_tria(nx, 2 * nx, Aug, Dn);
    for (int i = 0; i < nx; ++i)
        g[i] = Eg[i] + gi[i];
    memcpy(E, EE, sizeof(double) * (size_t)(nx * nx));
    memcpy(D, Dn, sizeof(double) * (size_t)(nx * nx));
}

/* Standard (covariance) combination of Table 3, left column. */
void or_filter_combine_cov(int nx, const double *Ai, const double *bi, const double *Ci,
                           const double *etai, const double *Ji, const double *Aj,
                           const double *bj, const double *Cj, const double *etaj,
                           const double *Jj, double *A, double *b, double *C, double *eta,
                           double *J)
{
    /* M = (I + C_i J_j)^{-1}, computed by Gauss-Jordan elimination */
    double T[OR_MAXD * OR_MAXD], M[OR_MAXD * OR_MAXD];
    mat_mul(nx, nx, nx, Ci, Jj, T);
    for (int i = 0; i < nx; ++i)
        T[i * nx + i] += 1.0;
    double aug[OR_MAXD * OR_MAXD * 2];
    int w = 2 * nx;
    for (int i = 0; i < nx; ++i)
        for (int t = 0; t < nx; ++t) {
            aug[i * w + t] = T[i * nx + t];
            aug[i * w + nx + t] = (i == t) ? 1.0 : 0.0;
        }
    for (int col = 0; col < nx; ++col) {
        int piv = col;
        for (int i = col + 1; i < nx; ++i)
            if (fabs(aug[i * w + col]) > fabs(aug[piv * w + col]))
                piv = i;
        if (piv != col)
            for (int t = 0; t < w; ++t) {
                double s = aug[col * w + t];
                aug[col * w + t] = aug[piv * w + t];
                aug[piv * w + t] = s;
            }
        double p = aug[col * w + col];
        for (int t = 0; t < w; ++t)
            aug[col * w + t] /= p;
        for (int i = 0; i < nx; ++i)
            if (i != col) {
                double f = aug[i * w + col];
                for (int t = 0; t < w; ++t)
                    aug[i * w + t] -= f * aug[col * w + t];
            }
    }
    for (int i = 0; i < nx; ++i)
        for (int t = 0; t < nx; ++t)
            M[i * nx + t] = aug[i * w + nx + t];
    double AjM[OR_MAXD * OR_MAXD], Mt[OR_MAXD * OR_MAXD];
    mat_mul(nx, nx, nx, Aj, M, AjM);
    mat_mul(nx, nx, nx, AjM, Ai, A);
    double Ceta[OR_MAXD], tmp[OR_MAXD], tb[OR_MAXD];
    mat_vec(nx, nx, Ci, etaj, Ceta);
    for (int i = 0; i < nx; ++i)
        tmp[i] = bi[i] + Ceta[i];
    mat_vec(nx, nx, AjM, tmp, tb);
    for (int i = 0; i < nx; ++i)
        b[i] = tb[i] + bj[i];
    double AMC[OR_MAXD * OR_MAXD], Cn[OR_MAXD * OR_MAXD];
    mat_mul(nx, nx, nx, AjM, Ci, AMC);
    mat_mult(nx, nx, nx, AMC, Aj, Cn);
    for (int i = 0; i < nx * nx; ++i)
        C[i] = Cn[i] + Cj[i];
    /* (I + J_j C_i)^{-1} = M^T since C_i, J_j are symmetric */
    mat_transpose(nx, nx, M, Mt);
    double Jb[OR_MAXD], r[OR_MAXD], Mr[OR_MAXD], Ar[OR_MAXD];
    mat_vec(nx, nx, Jj, bi, Jb);
    for (int i = 0; i < nx; ++i)
        r[i] = etaj[i] - Jb[i];
    mat_vec(nx, nx, Mt, r, Mr);
    mat_tvec(nx, nx, Ai, Mr, Ar);
    for (int i = 0; i < nx; ++i)
        eta[i] = Ar[i] + etai[i];
    double MJ[OR_MAXD * OR_MAXD], MJA[OR_MAXD * OR_MAXD], Jn[OR_MAXD * OR_MAXD];
    mat_mul(nx, nx, nx, Mt, Jj, MJ);
    mat_mul(nx, nx, nx, MJ, Ai, MJA);
    mat_tmul(nx, nx, nx, Ai, MJA, Jn);
    for (int i = 0; i < nx * nx; ++i)
        J[i] = Jn[i] + Ji[i];
}

/* ------------------------------------------------------------------------ */
/* First-order Taylor linearisation (Section 4.2: the iterated extended     */
/* smoother): F = Jacobian of f at the nominal mean, c = f(m) - F m,        */
/* Lambda = Q; H = Jacobian of h at the nominal mean, d = h(m) - H m,       */
/* Omega = R.  The nominal covariance is not used.                          */
/* ------------------------------------------------------------------------ */
/* d/dw of s1 = sin(w dt)/w and s2 = (1 - cos(w dt))/w, a = w dt:          */
/*   ds1 = dt^2 (a cos a - sin a)/a^2,  ds2 = dt^2 (a sin a - 1 + cos a)/a^2 */
/* with their Taylor series in a near 0 (-a/3 + a^3/30, 1/2 - a^2/8 + a^4/144)*/
static void ct_ds(double dt, double w, double *ds1, double *ds2)
{
    double a = w * dt;
    if (fabs(a) < 1e-3) {
        *ds1 = dt * dt * (-a / 3.0 + a * a * a / 30.0);
        *ds2 = dt * dt * (0.5 - a * a / 8.0 + a * a * a * a / 144.0);
    } else {
        *ds1 = dt * dt * (a * cos(a) - sin(a)) / (a * a);
        *ds2 = dt * dt * (a * sin(a) - 1.0 + cos(a)) / (a * a);
    }
}

/* Jacobian of the CT transition mean (5 x 5, row-major) */
void or_ct_jac_f(const double *prm, const double *x, double *J)
{
    double dt = prm[0], w = x[4], a = w * dt;
    double s1 = dt * sinc_(a), s2 = dt * 0.5 * a * sinc_(0.5 * a) * sinc_(0.5 * a);
    double ca = cos(a), sa = sin(a), ds1, ds2, vx = x[2], vy = x[3];
    ct_ds(dt, w, &ds1, &ds2);
    for (int i = 0; i < 25; ++i)
        J[i] = 0.0;
    J[0 * 5 + 0] = 1.0;
    J[0 * 5 + 2] = s1;
    J[0 * 5 + 3] = -s2;
    J[0 * 5 + 4] = ds1 * vx - ds2 * vy;
    J[1 * 5 + 1] = 1.0;
    J[1 * 5 + 2] = s2;
    J[1 * 5 + 3] = s1;
    J[1 * 5 + 4] = ds2 * vx + ds1 * vy;
    J[2 * 5 + 2] = ca;
    J[2 * 5 + 3] = -sa;
    J[2 * 5 + 4] = dt * (-sa * vx - ca * vy);
    J[3 * 5 + 2] = sa;
    J[3 * 5 + 3] = ca;
    J[3 * 5 + 4] = dt * (ca * vx - sa * vy);
    J[4 * 5 + 4] = 1.0;
}

/* Jacobian of the two bearings (2 x 5, row-major) */
void or_ct_jac_h(const double *prm, const double *x, double *J)
{
    for (int i = 0; i < 10; ++i)
        J[i] = 0.0;
    for (int s = 0; s < 2; ++s) {
        double dx = x[0] - prm[4 + 2 * s], dy = x[1] - prm[5 + 2 * s];
        double r2 = dx * dx + dy * dy;
        J[s * 5 + 0] = -dy / r2;
        J[s * 5 + 1] = dx / r2;
    }
}

/* ------------------------------------------------------------------------ */
/* CT model: per-step cubature linearisation (Section 4.1 / 4.3) at a       */
/* nominal trajectory (ms, Ns), k = 0..n.  Transition parameters of slot j  */
/* come from the marginal at j, measurement parameters of slot j (for       */
/* y_{j+1}) from the marginal at j+1.                                       */
/* ------------------------------------------------------------------------ */
int or_ct_linearize(int n, const double *prm, const double *ms, const double *Ns,
                    const double *y, int literal, double *F, double *c, double *SL, double *H,
                    double *d, double *SO)
{
    const int nx = 5, ny = 2;
    double Q[25], LQ[25], SOn[4] = {prm[3], 0.0, 0.0, prm[3]};
    or_ct_Q(prm, Q);
    if (or_cholesky(nx, Q, LQ) != 0)
        return -1;
    int bad = 0;
    if (literal == 2) { /* first-order Taylor (extended) */
        for (int j = 0; j < n; ++j) {
            const double *m = ms + (long)j * nx, *m1 = ms + (long)(j + 1) * nx;
            double fm[5], hm[2];
            double *Fj = F + (long)j * 25, *Hj = H + (long)j * 10;
            or_ct_f(prm, m, fm);
            or_ct_jac_f(prm, m, Fj);
            for (int r = 0; r < nx; ++r) {
                double s = fm[r];
                for (int q = 0; q < nx; ++q)
                    s -= Fj[r * nx + q] * m[q];
                c[(long)j * nx + r] = s;
            }
            memcpy(SL + (long)j * 25, LQ, sizeof(LQ));
            or_ct_h(prm, m1, y + (long)j * ny, hm);
            or_ct_jac_h(prm, m1, Hj);
            for (int r = 0; r < ny; ++r) {
                double s = hm[r];
                for (int q = 0; q < nx; ++q)
                    s -= Hj[r * nx + q] * m1[q];
                d[(long)j * ny + r] = s;
            }
            memcpy(SO + (long)j * 4, SOn, sizeof(SOn));
        }
        return 0;
    }
    if (literal == OR_RULE) { /* the installed sigma-point rule */
        if (g_rule_nx != nx)
            return -1;
        const int np = g_rule_np;
        double *X = malloc(sizeof(double) * (size_t)np * nx);
        double *Z = malloc(sizeof(double) * (size_t)np * nx);
        for (int j = 0; j < n; ++j) {
            const double *m = ms + (long)j * nx, *N = Ns + (long)j * nx * nx;
            rule_points(nx, m, N, X);
            for (int i = 0; i < np; ++i)
                or_ct_f(prm, X + (long)i * nx, Z + (long)i * nx);
            or_slr_rule(nx, nx, np, X, g_rule_w, m, N, Z, NULL, LQ, 0, F + (long)j * 25,
                        c + (long)j * 5, SL + (long)j * 25);
            const double *m1 = ms + (long)(j + 1) * nx, *N1 = Ns + (long)(j + 1) * nx * nx;
            rule_points(nx, m1, N1, X);
            for (int i = 0; i < np; ++i)
                or_ct_h(prm, X + (long)i * nx, y + (long)j * ny, Z + (long)i * ny);
            or_slr_rule(nx, ny, np, X, g_rule_w, m1, N1, Z, NULL, SOn, 0, H + (long)j * 10,
                        d + (long)j * 2, SO + (long)j * 4);
        }
        free(X);
        free(Z);
        return 0;
    }
    for (int j = 0; j < n; ++j) {
        double Xp[25], Xm[25], Zp[25], Zm[25], Yp[10], Ym[10];
        const double *m = ms + (long)j * nx, *N = Ns + (long)j * nx * nx;
        or_sigma_points(nx, m, N, Xp, Xm);
        for (int i = 0; i < nx; ++i) {
            or_ct_f(prm, Xp + i * nx, Zp + i * nx);
            or_ct_f(prm, Xm + i * nx, Zm + i * nx);
        }
        if (literal)
            bad += or_slr_literal(nx, nx, m, N, Zp, Zm, LQ, F + (long)j * 25, c + (long)j * 5,
                                  SL + (long)j * 25);
        else
            or_slr_residual(nx, nx, m, N, Zp, Zm, LQ, F + (long)j * 25, c + (long)j * 5,
                            SL + (long)j * 25);
        const double *m1 = ms + (long)(j + 1) * nx, *N1 = Ns + (long)(j + 1) * nx * nx;
        const double *yj = y + (long)j * ny;
        or_sigma_points(nx, m1, N1, Xp, Xm);
        for (int i = 0; i < nx; ++i) {
            or_ct_h(prm, Xp + i * nx, yj, Yp + i * ny);
            or_ct_h(prm, Xm + i * nx, yj, Ym + i * ny);
        }
        if (literal)
            bad += or_slr_literal(nx, ny, m1, N1, Yp, Ym, SOn, H + (long)j * 10, d + (long)j * 2,
                                  SO + (long)j * 4);
        else
            or_slr_residual(nx, ny, m1, N1, Yp, Ym, SOn, H + (long)j * 10, d + (long)j * 2,
                            SO + (long)j * 4);
    }
    return bad;
}

/* Algorithm 3 for the CT model (sequential in k; the parallel method      */
/* reaches the same marginals).  ms/Ns hold the initial nominal on entry    */
/* and the final one on exit; optional hist_* receive every pass's nominal  */
/* ([M][n+1][...]) and last_mf/last_Nf the filter output of the last pass.  */
int or_ct_ipls(int n, const double *prm, const double *m0, const double *N0, const double *y,
               int M, double *ms, double *Ns, double *hist_ms, double *hist_Ns, double *last_mf,
               double *last_Nf, int method)
{
    const int nx = 5, ny = 2;
    size_t nst = (size_t)(n + 1);
    double *F = malloc(sizeof(double) * (size_t)n * 25), *c = malloc(sizeof(double) * (size_t)n * 5);
    double *SL = malloc(sizeof(double) * (size_t)n * 25), *H = malloc(sizeof(double) * (size_t)n * 10);
    double *d = malloc(sizeof(double) * (size_t)n * 2), *SO = malloc(sizeof(double) * (size_t)n * 4);
    double *mf = malloc(sizeof(double) * nst * 5), *Nf = malloc(sizeof(double) * nst * 25);
    int rc = 0;
    for (int it = 0; it < M && rc == 0; ++it) {
        if (or_ct_linearize(n, prm, ms, Ns, y, method, F, c, SL, H, d, SO) != 0) {
            rc = -1;
            break;
        }
        or_sqrt_filter(n, nx, ny, m0, N0, F, c, SL, H, d, SO, 1, y, mf, Nf, NULL);
        or_sqrt_smoother(n, nx, F, c, SL, 1, mf, Nf, ms, Ns, NULL);
        if (hist_ms)
            memcpy(hist_ms + (size_t)it * nst * 5, ms, sizeof(double) * nst * 5);
        if (hist_Ns)
            memcpy(hist_Ns + (size_t)it * nst * 25, Ns, sizeof(double) * nst * 25);
    }
    if (last_mf)
        memcpy(last_mf, mf, sizeof(double) * nst * 5);
    if (last_Nf)
        memcpy(last_Nf, Nf, sizeof(double) * nst * 25);
    free(F); free(c); free(SL); free(H); free(d); free(SO); free(mf); free(Nf);
    return rc;
}

/* Pseudo-log-likelihood (Section 5.1) of the CT model linearised at the    */
/* given nominal: sum over k of log N(y_k; predicted mean, covariance).     */
/* ell (optional, [n]) receives the per-step terms.                          */
double or_ct_loglik(int n, const double *prm, const double *m0, const double *N0,
                    const double *y, const double *ms, const double *Ns, double *ell, int method)
{
    const int nx = 5, ny = 2;
    size_t nst = (size_t)(n + 1);
    double *F = malloc(sizeof(double) * (size_t)n * 25), *c = malloc(sizeof(double) * (size_t)n * 5);
    double *SL = malloc(sizeof(double) * (size_t)n * 25), *H = malloc(sizeof(double) * (size_t)n * 10);
    double *d = malloc(sizeof(double) * (size_t)n * 2), *SO = malloc(sizeof(double) * (size_t)n * 4);
    double *mf = malloc(sizeof(double) * nst * 5), *Nf = malloc(sizeof(double) * nst * 25);
    double *l = malloc(sizeof(double) * (size_t)n);
    double total = NAN;
    if (or_ct_linearize(n, prm, ms, Ns, y, method, F, c, SL, H, d, SO) == 0) {
        or_sqrt_filter(n, nx, ny, m0, N0, F, c, SL, H, d, SO, 1, y, mf, Nf, l);
        total = 0.0;
        for (int j = 0; j < n; ++j)
            total += l[j];
        if (ell)
            memcpy(ell, l, sizeof(double) * (size_t)n);
    }
    free(F); free(c); free(SL); free(H); free(d); free(SO); free(mf); free(Nf); free(l);
    return total;
}

/* ------------------------------------------------------------------------ */
/* Score of a linear-Gaussian model by Fisher's identity: the gradient of   */
/* log p(y) equals the posterior expectation of the complete-data score.    */
/* For step slot j it returns the symmetric sensitivities                   */
/*   Lbar_j = 1/2 Lam^{-1} (Sig_j - Lam) Lam^{-1},                          */
/*   Sig_j  = E[(x_{j+1} - F x_j - c)(...)^T | y_{1:n}],                    */
/*   Obar_j = 1/2 Om^{-1} (Sig'_j - Om) Om^{-1},                            */
/*   Sig'_j = E[(y_{j+1} - H x_{j+1} - d)(...)^T | y_{1:n}],                */
/* so that d log p / d theta = sum_j tr(Lbar_j dLam_j) + tr(Obar_j dOm_j).   */
/* Computed with covariance-form filter/smoother moments (independent of    */
/* any scan).  Returns the log-likelihood.                                  */
/* ------------------------------------------------------------------------ */
double or_lgssm_score_terms(int n, int nx, int ny, const double *m0, const double *P0,
                            const double *F, const double *c, const double *Lam, const double *H,
                            const double *d, const double *Om, long gstride, const double *y,
                            double *Lbar, double *Obar)
{
    size_t nst = (size_t)(n + 1);
    double *mf = malloc(sizeof(double) * nst * nx), *Pf = malloc(sizeof(double) * nst * nx * nx);
    double *ms = malloc(sizeof(double) * nst * nx), *Ps = malloc(sizeof(double) * nst * nx * nx);
    double *G = malloc(sizeof(double) * (size_t)n * nx * nx);
    double *l = malloc(sizeof(double) * (size_t)n);
    double total = NAN;
    if (or_cov_filter(n, nx, ny, m0, P0, F, c, Lam, H, d, Om, gstride, y, mf, Pf, NULL, NULL, l) == 0 &&
        or_cov_smoother(n, nx, F, c, Lam, gstride, mf, Pf, ms, Ps, G) == 0) {
        total = 0.0;
        for (int j = 0; j < n; ++j)
            total += l[j];
        for (int j = 0; j < n; ++j) {
            long g = gstride * j;
            const double *Fj = F + g * nx * nx, *cj = c + g * nx, *Lj = Lam + g * nx * nx;
            const double *Hj = H + g * ny * nx, *dj = d + g * ny, *Oj = Om + g * ny * ny;
            const double *mk = ms + (size_t)j * nx, *mk1 = ms + (size_t)(j + 1) * nx;
            const double *Pk = Ps + (size_t)j * nx * nx, *Pk1 = Ps + (size_t)(j + 1) * nx * nx;
            const double *Gk = G + (size_t)j * nx * nx;
            /* cross-covariance Cov(x_{j+1}, x_j | y) = P^s_{j+1} G_j^T */
            double Cx[OR_MAXD * OR_MAXD], T1[OR_MAXD * OR_MAXD], T2[OR_MAXD * OR_MAXD];
            double Sig[OR_MAXD * OR_MAXD], r[OR_MAXD], Fm[OR_MAXD];
            mat_mult(nx, nx, nx, Pk1, Gk, Cx);
            mat_vec(nx, nx, Fj, mk, Fm);
            for (int i = 0; i < nx; ++i)
                r[i] = mk1[i] - Fm[i] - cj[i];
            mat_mult(nx, nx, nx, Fj, Cx, T1); /* F Cx^T */
            mat_mul(nx, nx, nx, Fj, Pk, T2);
            double FPF[OR_MAXD * OR_MAXD];
            mat_mult(nx, nx, nx, T2, Fj, FPF);
            for (int a = 0; a < nx; ++a)
                for (int b = 0; b < nx; ++b)
                    Sig[a * nx + b] = r[a] * r[b] + Pk1[a * nx + b] - T1[a * nx + b] -
                                      T1[b * nx + a] + FPF[a * nx + b];
            /* Lbar = 1/2 Lam^{-1} (Sig - Lam) Lam^{-1} */
            double LL[OR_MAXD * OR_MAXD], X[OR_MAXD * OR_MAXD], Y[OR_MAXD * OR_MAXD], Z[OR_MAXD * OR_MAXD];
            if (or_cholesky(nx, Lj, LL) != 0) {
                total = NAN;
                break;
            }
            for (int i = 0; i < nx * nx; ++i)
                X[i] = Sig[i] - Lj[i];
            solve_lower(nx, LL, nx, X, Y);
            solve_lower_t(nx, LL, nx, Y, Z); /* Z = Lam^{-1} X */
            mat_transpose(nx, nx, Z, Y);     /* Y = X Lam^{-1} (X symmetric) -> (Lam^{-1} X)^T */
            solve_lower(nx, LL, nx, Y, X);
            solve_lower_t(nx, LL, nx, X, Z); /* Z = Lam^{-1} X Lam^{-1} */
            for (int i = 0; i < nx * nx; ++i)
                Lbar[(size_t)j * nx * nx + i] = 0.5 * Z[i];
            /* measurement part at state j+1 */
            double v[OR_MAXD], Hm[OR_MAXD], HP[OR_MAXD * OR_MAXD], HPH[OR_MAXD * OR_MAXD];
            double SigO[OR_MAXD * OR_MAXD], LO[OR_MAXD * OR_MAXD];
            mat_vec(ny, nx, Hj, mk1, Hm);
            for (int i = 0; i < ny; ++i)
                v[i] = y[(size_t)j * ny + i] - Hm[i] - dj[i];
            mat_mul(ny, nx, nx, Hj, Pk1, HP);
            mat_mult(ny, nx, ny, HP, Hj, HPH);
            for (int a = 0; a < ny; ++a)
                for (int b = 0; b < ny; ++b)
                    SigO[a * ny + b] = v[a] * v[b] + HPH[a * ny + b] - Oj[a * ny + b];
            if (or_cholesky(ny, Oj, LO) != 0) {
                total = NAN;
                break;
            }
            solve_lower(ny, LO, ny, SigO, Y);
            solve_lower_t(ny, LO, ny, Y, Z);
            mat_transpose(ny, ny, Z, Y);
            solve_lower(ny, LO, ny, Y, X);
            solve_lower_t(ny, LO, ny, X, Z);
            for (int i = 0; i < ny * ny; ++i)
                Obar[(size_t)j * ny * ny + i] = 0.5 * Z[i];
        }
    }
    free(mf); free(Pf); free(ms); free(Ps); free(G); free(l);
    return total;
}

/* CT model: gradient of the pseudo-log-likelihood at a frozen nominal with */
/* respect to theta = (log q1, log q2, log sigma).  With the nominal fixed, */
/* Lam_j = Q(theta) + R_j R_j^T and Om_j = sigma^2 I + R'_j R'_j^T, so       */
/* dLam/dlog q1 = q1 Qv, dLam/dlog q2 = q2 Qw and dOm/dlog sigma = 2 s^2 I.  */
double or_ct_score(int n, const double *prm, const double *m0, const double *N0,
                   const double *y, const double *ms, const double *Ns, double *grad3, int method)
{
    const int nx = 5, ny = 2;
    double *F = malloc(sizeof(double) * (size_t)n * 25), *c = malloc(sizeof(double) * (size_t)n * 5);
    double *SL = malloc(sizeof(double) * (size_t)n * 25), *H = malloc(sizeof(double) * (size_t)n * 10);
    double *d = malloc(sizeof(double) * (size_t)n * 2), *SO = malloc(sizeof(double) * (size_t)n * 4);
    double *Lam = malloc(sizeof(double) * (size_t)n * 25), *Om = malloc(sizeof(double) * (size_t)n * 4);
    double *Lbar = malloc(sizeof(double) * (size_t)n * 25), *Obar = malloc(sizeof(double) * (size_t)n * 4);
    double total = NAN;
    grad3[0] = grad3[1] = grad3[2] = NAN;
    if (or_ct_linearize(n, prm, ms, Ns, y, method, F, c, SL, H, d, SO) == 0) {
        for (int j = 0; j < n; ++j) {
            mat_mult(nx, nx, nx, SL + (size_t)j * 25, SL + (size_t)j * 25, Lam + (size_t)j * 25);
            mat_mult(ny, ny, ny, SO + (size_t)j * 4, SO + (size_t)j * 4, Om + (size_t)j * 4);
        }
        double P0[25];
        mat_mult(nx, nx, nx, N0, N0, P0);
        total = or_lgssm_score_terms(n, nx, ny, m0, P0, F, c, Lam, H, d, Om, 1, y, Lbar, Obar);
        double dQ1[25], dQ2[25], unit[8];
        memcpy(unit, prm, sizeof(unit));
        unit[1] = prm[1];
        unit[2] = 0.0;
        or_ct_Q(unit, dQ1); /* q1 * Qv */
        unit[1] = 0.0;
        unit[2] = prm[2];
        or_ct_Q(unit, dQ2); /* q2 * Qw */
        double g1 = 0.0, g2 = 0.0, g3 = 0.0, s2 = 2.0 * prm[3] * prm[3];
        for (int j = 0; j < n; ++j) {
            const double *Lb = Lbar + (size_t)j * 25, *Ob = Obar + (size_t)j * 4;
            for (int i = 0; i < 25; ++i) {
                g1 += Lb[i] * dQ1[i];
                g2 += Lb[i] * dQ2[i];
            }
            g3 += s2 * (Ob[0] + Ob[3]);
        }
        grad3[0] = g1;
        grad3[1] = g2;
        grad3[2] = g3;
    }
    free(F); free(c); free(SL); free(H); free(d); free(SO); free(Lam); free(Om); free(Lbar); free(Obar);
    return total;
}

/* ------------------------------------------------------------------------ */
/* Ricker population model with Poisson counts (Section 6.1):               */
/*   x_k = log a + x_{k-1} - exp(x_{k-1}) + q_k,   q_k ~ N(0, Q),           */
/*   y_k | x_k ~ Poisson(b exp(x_k)),  so E[y|x] = V[y|x] = b exp(x).       */
/* prm layout: a, b, Q.  The measurement noise is not additive: its         */
/* conditional variance enters Omega through the E[V[y|x]] term of the GSLR */
/* moments (Section 2.3).                                                    */
/* method 2: first-order Taylor (Section 4.2): F = 1 - exp(m),              */
/*   c = f(m) - F m, S_Lambda = sqrt(Q); H = b exp(m), d = b exp(m) - H m,  */
/*   S_Omega = sqrt(V[y|x](m)) = sqrt(b exp(m));                            */
/* method OR_RULE: the installed sigma-point rule (Section 4.3).            */
/* ------------------------------------------------------------------------ */
double or_ricker_f(const double *prm, double x) { return log(prm[0]) + x - exp(x); }

int or_ricker_linearize(int n, const double *prm, const double *ms, const double *Ns,
                        const double *y, int method, double *F, double *c, double *SL, double *H,
                        double *d, double *SO)
{
    (void)y;
    const double b = prm[1], sq = sqrt(prm[2]);
    if (method == 2) {
        for (int j = 0; j < n; ++j) {
            const double m = ms[j], m1 = ms[j + 1];
            F[j] = 1.0 - exp(m);
            c[j] = or_ricker_f(prm, m) - F[j] * m;
            SL[j] = sq;
            H[j] = b * exp(m1);
            d[j] = b * exp(m1) - H[j] * m1;
            SO[j] = sqrt(b * exp(m1));
        }
        return 0;
    }
    if (method != OR_RULE || g_rule_nx != 1)
        return -1;
    const int np = g_rule_np;
    double *X = malloc(sizeof(double) * (size_t)np), *Z = malloc(sizeof(double) * (size_t)np);
    double *Sg = malloc(sizeof(double) * (size_t)np);
    for (int j = 0; j < n; ++j) {
        rule_points(1, ms + j, Ns + j, X);
        for (int i = 0; i < np; ++i)
            Z[i] = or_ricker_f(prm, X[i]);
        or_slr_rule(1, 1, np, X, g_rule_w, ms + j, Ns + j, Z, NULL, &sq, 0, F + j, c + j, SL + j);
        rule_points(1, ms + j + 1, Ns + j + 1, X);
        for (int i = 0; i < np; ++i) {
            Z[i] = b * exp(X[i]);
            Sg[i] = sqrt(Z[i]);
        }
        or_slr_rule(1, 1, np, X, g_rule_w, ms + j + 1, Ns + j + 1, Z, Sg, NULL, 0, H + j, d + j,
                    SO + j);
    }
    free(X);
    free(Z);
    free(Sg);
    return 0;
}

/* Algorithm 3 for the Ricker model (sequential square-root filter and     */
/* smoother on each pass's linearisation); arguments as or_ct_ipls.        */
int or_ricker_ipls(int n, const double *prm, const double *m0, const double *N0,
                   const double *y, int M, double *ms, double *Ns, double *hist_ms,
                   double *hist_Ns, double *last_mf, double *last_Nf, int method)
{
    size_t nst = (size_t)(n + 1);
    double *G = malloc(sizeof(double) * (size_t)n * 6), *mf = malloc(sizeof(double) * nst);
    double *Nf = malloc(sizeof(double) * nst);
    double *F = G, *c = G + n, *SL = G + 2 * n, *H = G + 3 * n, *d = G + 4 * n, *SO = G + 5 * n;
    int rc = 0;
    for (int it = 0; it < M && rc == 0; ++it) {
        if (or_ricker_linearize(n, prm, ms, Ns, y, method, F, c, SL, H, d, SO) != 0) {
            rc = -1;
            break;
        }
        or_sqrt_filter(n, 1, 1, m0, N0, F, c, SL, H, d, SO, 1, y, mf, Nf, NULL);
        or_sqrt_smoother(n, 1, F, c, SL, 1, mf, Nf, ms, Ns, NULL);
        if (hist_ms)
            memcpy(hist_ms + (size_t)it * nst, ms, sizeof(double) * nst);
        if (hist_Ns)
            memcpy(hist_Ns + (size_t)it * nst, Ns, sizeof(double) * nst);
    }
    if (last_mf)
        memcpy(last_mf, mf, sizeof(double) * nst);
    if (last_Nf)
        memcpy(last_Nf, Nf, sizeof(double) * nst);
    free(G);
    free(mf);
    free(Nf);
    return rc;
}

/* Pseudo-log-likelihood (Section 5.1) of the Ricker model linearised at    */
/* the given nominal; ell (optional, [n]) receives the per-step terms.      */
double or_ricker_loglik(int n, const double *prm, const double *m0, const double *N0,
                        const double *y, const double *ms, const double *Ns, double *ell,
                        int method)
{
    size_t nst = (size_t)(n + 1);
    double *G = malloc(sizeof(double) * (size_t)n * 6), *mf = malloc(sizeof(double) * nst);
    double *Nf = malloc(sizeof(double) * nst), *l = malloc(sizeof(double) * (size_t)n);
    double *F = G, *c = G + n, *SL = G + 2 * n, *H = G + 3 * n, *d = G + 4 * n, *SO = G + 5 * n;
    double total = NAN;
    if (or_ricker_linearize(n, prm, ms, Ns, y, method, F, c, SL, H, d, SO) == 0) {
        or_sqrt_filter(n, 1, 1, m0, N0, F, c, SL, H, d, SO, 1, y, mf, Nf, l);
        total = 0.0;
        for (int j = 0; j < n; ++j)
            total += l[j];
        if (ell)
            memcpy(ell, l, sizeof(double) * (size_t)n);
    }
    free(G);
    free(mf);
    free(Nf);
    free(l);
    return total;
}

/* ------------------------------------------------------------------------ */
/* Batches of independent sequences (OpenMP over sequences).               */
/* y_off[B+1]: measurement offsets; sequence b has n_b = y_off[b+1]-y_off[b]*/
/* steps and states at x_off[b] = y_off[b] + b.                              */
/* ------------------------------------------------------------------------ */
int or_ct_ipls_batch(int B, const long *y_off, const double *prm, const double *m0,
                     const double *N0, const double *y, int M, double *ms, double *Ns)
{
    int rc = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : rc)
    for (int b = 0; b < B; ++b) {
        long n = y_off[b + 1] - y_off[b];
        long xo = y_off[b] + b;
        rc |= or_ct_ipls((int)n, prm, m0, N0, y + y_off[b] * 2, M, ms + xo * 5, Ns + xo * 25,
                         NULL, NULL, NULL, NULL, 0);
    }
    return rc;
}

/* Linear model with one shared parameter set: square-root filter+smoother. */
int or_linear_smoother_batch(int B, const long *y_off, int nx, int ny, const double *m0,
                             const double *N0, const double *F, const double *c,
                             const double *SL, const double *H, const double *d,
                             const double *SO, const double *y, double *ms, double *Ns)
{
    int rc = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : rc)
    for (int b = 0; b < B; ++b) {
        long n = y_off[b + 1] - y_off[b];
        long xo = y_off[b] + b;
        double *mf = malloc(sizeof(double) * (size_t)(n + 1) * nx);
        double *Nf = malloc(sizeof(double) * (size_t)(n + 1) * nx * nx);
        rc |= or_sqrt_filter((int)n, nx, ny, m0, N0, F, c, SL, H, d, SO, 0, y + y_off[b] * ny,
                             mf, Nf, NULL);
        rc |= or_sqrt_smoother((int)n, nx, F, c, SL, 0, mf, Nf, ms + xo * nx, Ns + xo * nx * nx,
                               NULL);
        free(mf);
        free(Nf);
    }
    return rc;
}

int or_ct_loglik_batch(int B, const long *y_off, const double *prm, const double *m0,
                       const double *N0, const double *y, const double *ms, const double *Ns,
                       double *ll)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < B; ++b) {
        long n = y_off[b + 1] - y_off[b];
        long xo = y_off[b] + b;
        ll[b] = or_ct_loglik((int)n, prm, m0, N0, y + y_off[b] * 2, ms + xo * 5, Ns + xo * 25,
                             NULL, 0);
    }
    return 0;
}

int or_ct_score_batch(int B, const long *y_off, const double *prm, const double *m0,
                      const double *N0, const double *y, const double *ms, const double *Ns,
                      double *ll, double *grad3)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < B; ++b) {
        long n = y_off[b + 1] - y_off[b];
        long xo = y_off[b] + b;
        ll[b] = or_ct_score((int)n, prm, m0, N0, y + y_off[b] * 2, ms + xo * 5, Ns + xo * 25,
                            grad3 + 3 * b, 0);
    }
    return 0;
}

int or_max_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
