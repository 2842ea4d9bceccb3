/*
 * PDMCF reference oracle.  TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of the PDMCF method of Zhang & Boyd,
 * "Solving Large Multicommodity Network Flow Problems on GPUs" (arXiv 2501.17996).
 * It exists to check the HIP solver.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the HIP library, and the HIP library never calls it.
 *
 * Every step is written the way the paper states it, with explicit loops and
 * no blocking or fusion:
 *   - problem (e-prob)/(e-compact-prob), Section 1.1;
 *   - residual r(Q), eq. (e-res), Section 1.2;
 *   - reduced Lagrangian (e-L), Section 2.1 (used for the dual objective);
 *   - over-relaxed PDHG step, eq. (e-pdhg-step), Section 2.2;
 *   - the two proximal operators, Section 2.3;
 *   - adaptive primal weight, eq. (e-primal_weight), Section 2.4;
 *   - eta = 1/sqrt(2 d_max), eq. (e-eta) and Appendix A;
 *   - Algorithm 2.1 (PDMCF) with its initialization and stopping rule, Section 2.5;
 *   - the sort-based simplex projection of Section 2.6.
 *
 * Readings taken where the paper is silent (each is listed in the design notes):
 *   - the relative KKT residual, the Y that pairs with F^ in the gap (Y^k),
 *     k = 0 counting as a multiple of k_adapt, tau absolute, the stable form of
 *     the log prox for y > 0, bisection for the power prox, d_i = in+out degree;
 *   - the alpha-fair family u(s) = w s^{1-alpha}/(1-alpha), alpha > 0, alpha != 1, as the
 *     general strictly concave increasing utility of Section 1.1 whose one-dimensional
 *     prox Section 2.3 leaves to the general case (log is its limit alpha -> 1, the
 *     power utility w s^gamma is alpha = 1 - gamma with weight w gamma).
 *
 * Layout: F is n x m with F[l*n + i] the flow on edge l destined to node i.
 * Y, T, W are n x n with X[j*n + i] holding entry (i, j); w[j*n+i] weights the
 * traffic from j to i.  Edge l runs tail[l] -> head[l]; A[head,l]=+1, A[tail,l]=-1.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_UTIL_LOG 0
#define ORC_UTIL_POWER 1
#define ORC_UTIL_ALPHA 2

/* metric slots filled by orc_get_metrics */
enum {
    M_K = 0, M_OMEGA, M_ALPHA, M_BETA, M_DF, M_DY, M_R, M_RPAPER, M_RELP, M_RELD, M_RELG,
    M_RELKKT, M_PRIMAL, M_DUAL, M_INFEAS, M_CHECKED, M_A, M_B, M_E, M_COUNT
};

typedef struct orc_solver {
    int32_t n, m;
    int32_t *tail, *head;
    double *cap;
    int32_t utility;
    double gamma;
    double *w;
    double rho, theta, tau, omega0, eta;
    int32_t k_adapt, nthreads;
    int64_t adapt_until; /* omega adapts only while k < adapt_until (< 0: always) */
    /* iterate state: F^{k-1/2}, Y^k, omega^k, step sizes, k */
    double *F, *Y;
    double omega, alpha, beta;
    int64_t k;
    /* work arrays */
    double *Q, *Fhat, *Fbar, *Fnew, *V, *Ynew, *That, *Up;
    double metrics[M_COUNT];
    int have_metrics;
} orc_solver;

/* ------------------------------------------------------------------ utilities */
/* Section 1.1 "Network utility": u(s) = w log s, u(s) = w s^gamma, or the alpha-fair
 * u(s) = w s^{1-a}/(1-a) (the parameter g is gamma for the power utility, a for alpha-fair). */
static double util_u(int32_t ut, double g, double w, double s)
{
    if (ut == ORC_UTIL_LOG) return w * log(s);
    if (ut == ORC_UTIL_POWER) return w * pow(s, g);
    return w * pow(s, 1.0 - g) / (1.0 - g);
}

/* derivative u'(s), used for U' in the residual (Section 1.2, "Optimality condition") */
static double util_du(int32_t ut, double g, double w, double s)
{
    if (ut == ORC_UTIL_LOG) return w / s;
    if (ut == ORC_UTIL_POWER) return w * g * pow(s, g - 1.0);
    return w * pow(s, -g);
}

/* the maximizer s of y s + u(s): the traffic that dual price y asks for (y < 0), from
 * u'(s) = -y */
static double util_traffic_of_price(int32_t ut, double g, double w, double y)
{
    if (ut == ORC_UTIL_LOG) return w / (-y);
    if (ut == ORC_UTIL_POWER) return pow(w * g / (-y), 1.0 / (1.0 - g));
    return pow(w / (-y), 1.0 / g);
}

/* conjugate (-u)^*(y) = sup_s ( y s + u(s) ), finite only for y < 0 (used in (e-L)).
 * log:         -w + w log w - w log(-y)
 * power:       (1/g - 1) (w g)^{1/(1-g)} (-y)^{-g/(1-g)}
 * alpha-fair:  at the maximizer s, w s^{1-a} = -y s, so the value is (-y) s a / (1 - a) */
static double util_conj(int32_t ut, double g, double w, double y)
{
    if (!(y < 0.0)) return INFINITY;
    if (ut == ORC_UTIL_LOG) return -w + w * log(w) - w * log(-y);
    if (ut == ORC_UTIL_POWER) return (1.0 / g - 1.0) * pow(w * g, 1.0 / (1.0 - g)) * pow(-y, -g / (1.0 - g));
    return (-y) * util_traffic_of_price(ut, g, w, y) * g / (1.0 - g);
}

/* ---------------------------------------------------------- proximal operators */
/* Section 2.3, "Second proximal operator", weighted log utility:
 * prox(y) = (y - sqrt(y^2 + 4 beta w)) / 2.  For y > 0 the equal form
 * -2 beta w / (y + sqrt(y^2 + 4 beta w)) avoids cancellation. */
double orc_prox_log(double y, double beta, double w)
{
    double s = sqrt(y * y + 4.0 * beta * w);
    if (y <= 0.0) return 0.5 * (y - s);
    return -2.0 * beta * w / (y + s);
}

/* Section 2.3, weighted power utility: prox(y) is the unique z < 0 with
 * (-z)^{c1+2} + y (-z)^{c1+1} - c1 c2 = 0, c1 = g/(1-g), c2 = beta (1/g - 1) (w g)^{1/(1-g)}.
 * Solved by bisection in t = -z on [a, a + (c1 c2)^{1/(c1+2)}], a = max(-y, 0),
 * down to adjacent doubles. */
static double power_poly(double t, double y, double c1, double k)
{
    return pow(t, c1 + 1.0) * (t + y) - k;
}

/* the root t > a = max(-y, 0) of t^{c1+1} (t + y) = k (k > 0), by bisection on
 * [a, a + k^{1/(c1+2)}] down to adjacent doubles */
static double bisect_root(double y, double c1, double k)
{
    double a = y < 0.0 ? -y : 0.0;
    double lo = a, hi = a + pow(k, 1.0 / (c1 + 2.0));
    int guard = 0;
    while (power_poly(hi, y, c1, k) < 0.0 && guard++ < 64) hi = a + 2.0 * (hi - a);
    for (int it = 0; it < 5000; ++it) {
        double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        if (power_poly(mid, y, c1, k) < 0.0) lo = mid; else hi = mid;
    }
    return fabs(power_poly(lo, y, c1, k)) < fabs(power_poly(hi, y, c1, k)) ? lo : hi;
}

double orc_prox_power(double y, double beta, double w, double g)
{
    double c1 = g / (1.0 - g);
    double c2 = beta * (1.0 / g - 1.0) * pow(w * g, 1.0 / (1.0 - g));
    return -bisect_root(y, c1, c1 * c2);
}

/* Alpha-fair utility u(s) = w s^{1-a}/(1-a): the optimality condition of the prox,
 * z + beta s(z) = y with the traffic s(z) = (w/(-z))^{1/a} of price z < 0, reads with
 * t = -z and p = 1/a:  t^{p+1} + y t^p = beta w^p.  Same bisection, with c1 = p - 1. */
double orc_prox_alpha(double y, double beta, double w, double a)
{
    double p = 1.0 / a;
    return -bisect_root(y, p - 1.0, beta * pow(w, p));
}

static double prox_dual(int32_t ut, double g, double y, double beta, double w)
{
    if (ut == ORC_UTIL_LOG) return orc_prox_log(y, beta, w);
    if (ut == ORC_UTIL_POWER) return orc_prox_power(y, beta, w, g);
    return orc_prox_alpha(y, beta, w, g);
}

/* ------------------------------------------------------ projection onto S_l */
static int cmp_desc(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) - (x > y);
}

/* Section 2.3 "First proximal operator" and Section 2.6 "Projection onto scaled
 * simplex": Pi(f) = (f - mu 1)_+ with mu the smallest nonnegative value such that
 * 1^T (f - mu 1)_+ <= c.  When 1^T (f)_+ > c, sort f descending into f', take
 * the largest t with f'_t - (sum_{i<=t} f'_i - c)/t > 0, and mu = (sum_{i<=t} f'_i - c)/t.
 * `work` holds n doubles.  Returns mu. */
static double project_column(int32_t n, const double *f, double c, double *out, double *work)
{
    double pos = 0.0;
    for (int32_t i = 0; i < n; ++i)
        if (f[i] > 0.0) pos += f[i];
    double mu = 0.0;
    if (pos > c) {
        memcpy(work, f, sizeof(double) * (size_t)n);
        qsort(work, (size_t)n, sizeof(double), cmp_desc);
        double s = 0.0;
        for (int32_t t = 1; t <= n; ++t) {
            s += work[t - 1];
            double cand = (s - c) / (double)t;
            if (work[t - 1] - cand > 0.0) mu = cand;
        }
    }
    for (int32_t i = 0; i < n; ++i) {
        double v = f[i] - mu;
        out[i] = v > 0.0 ? v : 0.0;
    }
    return mu;
}

double orc_project(int32_t n, const double *f, double c, double *out)
{
    double *work = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double mu = project_column(n, f, c, out, work);
    free(work);
    return mu;
}

/* -------------------------------------------------------------- step size eta */
/* Section 2.4, "A simple bound on ||A||_2": lambda_max(A A^T) <= 2 d_max with
 * d_i = (A A^T)_ii = in-degree + out-degree (Appendix A), so eta = 1/sqrt(2 d_max). */
double orc_eta(int32_t n, int32_t m, const int32_t *tail, const int32_t *head)
{
    int64_t *d = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    for (int32_t l = 0; l < m; ++l) {
        d[tail[l]] += 1;
        d[head[l]] += 1;
    }
    int64_t dmax = 0;
    for (int32_t i = 0; i < n; ++i)
        if (d[i] > dmax) dmax = d[i];
    free(d);
    return 1.0 / sqrt(2.0 * (double)dmax);
}

/* ------------------------------------------------------------ column kernels */
/* First two lines of (e-pdhg-step) and the F relaxation, for one edge column:
 * q = f + alpha (Y[:,head] - Y[:,tail]) (that is, column l of F + alpha Y A),
 * fhat = Pi_{S_l}(q), fbar = 2 fhat - f, fnew = rho fhat + (1 - rho) f. */
static double edge_column(int32_t n, const double *f, const double *yh, const double *yt, double alpha,
                          double c, double rho, double *q, double *fhat, double *fbar, double *fnew,
                          double *work)
{
    for (int32_t i = 0; i < n; ++i) q[i] = f[i] + alpha * (yh[i] - yt[i]);
    double mu = project_column(n, q, c, fhat, work);
    for (int32_t i = 0; i < n; ++i) {
        fbar[i] = 2.0 * fhat[i] - f[i];
        fnew[i] = rho * fhat[i] + (1.0 - rho) * f[i];
    }
    return mu;
}

double orc_edge_column(int32_t n, const double *f, const double *yh, const double *yt, double alpha,
                       double c, double rho, double *fhat, double *fbar, double *fnew)
{
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    double *work = (double *)malloc(sizeof(double) * (size_t)n);
    double mu = edge_column(n, f, yh, yt, alpha, c, rho, q, fhat, fbar, fnew, work);
    free(q);
    free(work);
    return mu;
}

/* Third and fifth lines of (e-pdhg-step) for node column j, given v = column j of
 * Fbar A^T:  yhat_i = prox(y_i - beta v_i) for i != j, yhat_j = 0 (Algorithm 2.1),
 * ynew = rho yhat + (1 - rho) y. */
static void node_column(int32_t n, int32_t j, const double *v, const double *y, const double *w,
                        double beta, double rho, int32_t ut, double g, double *yhat, double *ynew)
{
    for (int32_t i = 0; i < n; ++i) {
        double z = (i == j) ? 0.0 : prox_dual(ut, g, y[i] - beta * v[i], beta, w[i]);
        if (yhat) yhat[i] = z;
        ynew[i] = rho * z + (1.0 - rho) * y[i];
    }
}

/* Column j of Fbar A^T from the columns of the edges entering j (fbar_in, nin of
 * them, each n long) and leaving j (fbar_out): sum of entering minus sum of leaving. */
void orc_node_column(int32_t n, int32_t j, int32_t nin, const double *fbar_in, int32_t nout,
                     const double *fbar_out, const double *y, const double *w, double beta, double rho,
                     int32_t ut, double g, double *v_out, double *yhat, double *ynew)
{
    for (int32_t i = 0; i < n; ++i) v_out[i] = 0.0;
    for (int32_t e = 0; e < nin; ++e)
        for (int32_t i = 0; i < n; ++i) v_out[i] += fbar_in[(size_t)e * n + i];
    for (int32_t e = 0; e < nout; ++e)
        for (int32_t i = 0; i < n; ++i) v_out[i] -= fbar_out[(size_t)e * n + i];
    node_column(n, j, v_out, y, w, beta, rho, ut, g, yhat, ynew);
}

/* ------------------------------------------------------------------- solver */
static void *xcalloc(size_t count, size_t size)
{
    return calloc(count ? count : 1, size);
}

void orc_reset(orc_solver *s)
{
    /* Section 2.5, "Initialization": F^{-1/2} = 0, Y^0 = I - 1 1^T, omega^0, alpha, beta. */
    size_t nm = (size_t)s->n * s->m, nn = (size_t)s->n * s->n;
    memset(s->F, 0, sizeof(double) * nm);
    for (int32_t j = 0; j < s->n; ++j)
        for (int32_t i = 0; i < s->n; ++i) s->Y[(size_t)j * s->n + i] = (i == j) ? 0.0 : -1.0;
    (void)nn;
    s->omega = s->omega0;
    s->alpha = s->eta / s->omega;
    s->beta = s->eta * s->omega;
    s->k = 0;
    s->have_metrics = 0;
    for (int i = 0; i < M_COUNT; ++i) s->metrics[i] = NAN;
}

void orc_destroy(orc_solver *s)
{
    if (!s) return;
    free(s->tail); free(s->head); free(s->cap); free(s->w);
    free(s->F); free(s->Y); free(s->Q); free(s->Fhat); free(s->Fbar); free(s->Fnew);
    free(s->V); free(s->Ynew); free(s->That); free(s->Up);
    free(s);
}

orc_solver *orc_create(int32_t n, int32_t m, const int32_t *tail, const int32_t *head, const double *cap,
                       int32_t utility, double gamma, const double *w, double rho, double theta, double tau,
                       double omega0, int32_t k_adapt, int32_t nthreads, int64_t adapt_until)
{
    if (n < 2 || m < 1) return NULL;
    orc_solver *s = (orc_solver *)calloc(1, sizeof(orc_solver));
    size_t nm = (size_t)n * m, nn = (size_t)n * n;
    s->n = n; s->m = m;
    s->tail = (int32_t *)malloc(sizeof(int32_t) * m);
    s->head = (int32_t *)malloc(sizeof(int32_t) * m);
    s->cap = (double *)malloc(sizeof(double) * m);
    s->w = (double *)malloc(sizeof(double) * nn);
    memcpy(s->tail, tail, sizeof(int32_t) * m);
    memcpy(s->head, head, sizeof(int32_t) * m);
    memcpy(s->cap, cap, sizeof(double) * m);
    memcpy(s->w, w, sizeof(double) * nn);
    s->utility = utility; s->gamma = gamma;
    s->rho = rho; s->theta = theta; s->tau = tau; s->omega0 = omega0;
    s->k_adapt = k_adapt; s->nthreads = nthreads > 0 ? nthreads : 1;
    s->adapt_until = adapt_until;
    s->eta = orc_eta(n, m, tail, head);
    s->F = (double *)xcalloc(nm, sizeof(double));
    s->Q = (double *)xcalloc(nm, sizeof(double));
    s->Fhat = (double *)xcalloc(nm, sizeof(double));
    s->Fbar = (double *)xcalloc(nm, sizeof(double));
    s->Fnew = (double *)xcalloc(nm, sizeof(double));
    s->Y = (double *)xcalloc(nn, sizeof(double));
    s->V = (double *)xcalloc(nn, sizeof(double));
    s->Ynew = (double *)xcalloc(nn, sizeof(double));
    s->That = (double *)xcalloc(nn, sizeof(double));
    s->Up = (double *)xcalloc(nn, sizeof(double));
    if (!s->F || !s->Q || !s->Fhat || !s->Fbar || !s->Fnew || !s->Y || !s->V || !s->Ynew || !s->That ||
        !s->Up) {
        orc_destroy(s);
        return NULL;
    }
    orc_reset(s);
    return s;
}

/* Residual and KKT quantities for Q = Q^k and Fhat = Pi(Q), with the dual Y^k
 * that formed Q (Section 1.2 eq. (e-res); dual objective from (e-L)). */
static void residual(orc_solver *s)
{
    const int32_t n = s->n, m = s->m, ut = s->utility;
    const double g = s->gamma;
    double *T = s->That, *Up = s->Up;
    const double *Y = s->Y;
    /* T^ = -Fhat A^T: edge l adds Fhat[:,l] to column tail and removes it from column head. */
    memset(T, 0, sizeof(double) * (size_t)n * n);
    for (int32_t l = 0; l < m; ++l) {
        const double *f = s->Fhat + (size_t)l * n;
        double *th = T + (size_t)s->head[l] * n, *tt = T + (size_t)s->tail[l] * n;
        for (int32_t i = 0; i < n; ++i) {
            th[i] -= f[i];
            tt[i] += f[i];
        }
    }
    int64_t nonpos = 0;
    for (int32_t j = 0; j < n; ++j)
        for (int32_t i = 0; i < n; ++i)
            if (i != j && !(T[(size_t)j * n + i] > 0.0)) ++nonpos;
    int yfeas = 1;
    for (int32_t j = 0; j < n; ++j)
        for (int32_t i = 0; i < n; ++i)
            if (i != j && !(Y[(size_t)j * n + i] < 0.0)) yfeas = 0;

    double *M = s->metrics;
    M[M_INFEAS] = (double)nonpos / ((double)n * (double)(n - 1));
    /* e = ||Fhat - Q||^2, and the support term sum_l c_l (max_i (Y A)_{il})_+ */
    double e = 0.0, support = 0.0;
    for (int32_t l = 0; l < m; ++l) {
        const double *fh = s->Fhat + (size_t)l * n, *q = s->Q + (size_t)l * n;
        const double *yh = Y + (size_t)s->head[l] * n, *yt = Y + (size_t)s->tail[l] * n;
        double gmax = -INFINITY;
        for (int32_t i = 0; i < n; ++i) {
            double d = fh[i] - q[i];
            e += d * d;
            double ya = yh[i] - yt[i];
            if (ya > gmax) gmax = ya;
        }
        support += s->cap[l] * (gmax > 0.0 ? gmax : 0.0);
    }
    M[M_E] = e;
    double r = INFINITY, a = NAN, b = NAN, p = INFINITY;
    if (nonpos == 0) {
        /* U'_{ij} = u'_{ij}(T^_{ij}), U'_{ii} = 0; G = U' A, column l = U'[:,head] - U'[:,tail]. */
        p = 0.0;
        for (int32_t j = 0; j < n; ++j)
            for (int32_t i = 0; i < n; ++i) {
                size_t x = (size_t)j * n + i;
                if (i == j) {
                    Up[x] = 0.0;
                } else {
                    Up[x] = util_du(ut, g, s->w[x], T[x]);
                    p -= util_u(ut, g, s->w[x], T[x]);
                }
            }
        a = 0.0;
        b = 0.0;
        for (int32_t l = 0; l < m; ++l) {
            const double *uh = Up + (size_t)s->head[l] * n, *ut_ = Up + (size_t)s->tail[l] * n;
            const double *fh = s->Fhat + (size_t)l * n, *q = s->Q + (size_t)l * n;
            for (int32_t i = 0; i < n; ++i) {
                double G = uh[i] - ut_[i];
                a += G * G;
                b += G * (fh[i] - q[i]);
            }
        }
        /* eq. (e-res) */
        if (e > 0.0 && b >= 0.0) r = a - b * b / e;
        else r = a;
    }
    M[M_A] = a;
    M[M_B] = b;
    M[M_R] = r;
    M[M_RPAPER] = r / ((double)n * (double)m);
    M[M_RELD] = (nonpos == 0 && a > 0.0) ? sqrt((r > 0.0 ? r : 0.0) / a) : INFINITY;
    M[M_PRIMAL] = p;
    /* dual objective D(Y) = -sum_{i!=j} (-u_ij)^*(Y_ij) - sum_l c_l (max_i (YA)_il)_+ */
    double d = -INFINITY;
    double relp = INFINITY;
    if (yfeas) {
        double cs = 0.0, num = 0.0, den = 0.0;
        for (int32_t j = 0; j < n; ++j)
            for (int32_t i = 0; i < n; ++i) {
                if (i == j) continue;
                size_t x = (size_t)j * n + i;
                cs += util_conj(ut, g, s->w[x], Y[x]);
                double td = util_traffic_of_price(ut, g, s->w[x], Y[x]) - T[x];
                num += td * td;
                den += T[x] * T[x];
            }
        d = -cs - support;
        relp = den > 0.0 ? sqrt(num) / sqrt(den) : INFINITY;
    }
    M[M_DUAL] = d;
    M[M_RELP] = relp;
    double relg = (isfinite(p) && isfinite(d)) ? (p - d) / (1.0 + fabs(p) + fabs(d)) : INFINITY;
    M[M_RELG] = relg;
    double kkt = INFINITY;
    if (nonpos == 0 && yfeas) {
        kkt = M[M_RELP];
        if (M[M_RELD] > kkt) kkt = M[M_RELD];
        if (relg > kkt) kkt = relg;
    }
    M[M_RELKKT] = kkt;
    M[M_CHECKED] = 1.0;
}

/* One iteration of Algorithm 2.1: step 2 (the PDHG update (e-pdhg-step)) and
 * step 3 (the adaptive primal weight (e-primal_weight)).  With check != 0 the
 * residual r^{k+1} = r(Q^k) and the KKT quantities are computed as well. */
void orc_step(orc_solver *s, int32_t check)
{
    const int32_t n = s->n, m = s->m;
    const double alpha = s->alpha, beta = s->beta, rho = s->rho;
    /* Fhat^{k+1/2} = Pi(F^{k-1/2} + alpha Y^k A); Fbar^{k+1} = 2 Fhat - F; F^{k+1/2} relaxed */
#pragma omp parallel num_threads(s->nthreads)
    {
        double *work = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int32_t l = 0; l < m; ++l) {
            size_t o = (size_t)l * n;
            edge_column(n, s->F + o, s->Y + (size_t)s->head[l] * n, s->Y + (size_t)s->tail[l] * n, alpha,
                        s->cap[l], rho, s->Q + o, s->Fhat + o, s->Fbar + o, s->Fnew + o, work);
        }
        free(work);
    }
    /* V = Fbar A^T, accumulated edge by edge in ascending order */
    memset(s->V, 0, sizeof(double) * (size_t)n * n);
    for (int32_t l = 0; l < m; ++l) {
        const double *fb = s->Fbar + (size_t)l * n;
        double *vh = s->V + (size_t)s->head[l] * n, *vt = s->V + (size_t)s->tail[l] * n;
        for (int32_t i = 0; i < n; ++i) {
            vh[i] += fb[i];
            vt[i] -= fb[i];
        }
    }
    /* Yhat^{k+1} = prox(Y^k - beta V) off the diagonal, 0 on it; Y^{k+1} relaxed */
#pragma omp parallel for schedule(static) num_threads(s->nthreads)
    for (int32_t j = 0; j < n; ++j) {
        size_t o = (size_t)j * n;
        node_column(n, j, s->V + o, s->Y + o, s->w + o, beta, rho, s->utility, s->gamma, NULL, s->Ynew + o);
    }
    /* Delta_F = ||F^{k+1/2} - F^{k-1/2}||_F, Delta_Y = ||Y^{k+1} - Y^k||_F (Section 2.4) */
    double sf = 0.0, sy = 0.0;
    for (size_t x = 0; x < (size_t)n * m; ++x) {
        double d = s->Fnew[x] - s->F[x];
        sf += d * d;
    }
    for (size_t x = 0; x < (size_t)n * n; ++x) {
        double d = s->Ynew[x] - s->Y[x];
        sy += d * d;
    }
    double dF = sqrt(sf), dY = sqrt(sy);
    for (int i = M_R; i < M_COUNT; ++i) s->metrics[i] = NAN;
    s->metrics[M_CHECKED] = 0.0;
    if (check) residual(s); /* uses Q^k, Fhat^{k+1/2} and Y^k, before Y is replaced */
    /* accept the step */
    double *t = s->F; s->F = s->Fnew; s->Fnew = t;
    t = s->Y; s->Y = s->Ynew; s->Ynew = t;
    /* Algorithm 2.1 step 3: adapt omega when k is a multiple of k_adapt (k = 0 included)
     * and both step norms exceed tau; optionally only before iteration adapt_until, the
     * freeze Section 2.4 allows. */
    if (s->k_adapt > 0 && s->k % s->k_adapt == 0 && (s->adapt_until < 0 || s->k < s->adapt_until) &&
        dF > s->tau && dY > s->tau) {
        s->omega = pow(dY / dF, s->theta) * pow(s->omega, 1.0 - s->theta);
        s->alpha = s->eta / s->omega;
        s->beta = s->eta * s->omega;
    }
    s->k += 1;
    s->metrics[M_K] = (double)s->k;
    s->metrics[M_OMEGA] = s->omega;
    s->metrics[M_ALPHA] = s->alpha;
    s->metrics[M_BETA] = s->beta;
    s->metrics[M_DF] = dF;
    s->metrics[M_DY] = dY;
    s->have_metrics = check ? 1 : 0;
}

/* Algorithm 2.1 with its stopping test.  stop_rule 0: relative KKT <= tol;
 * stop_rule 1: the paper's r^k < n m tol.  The residual is evaluated every
 * check_every iterations and at the last allowed iteration.
 * Returns 1 converged, 2 iteration limit, 3 diverged (non-finite step norms). */
int32_t orc_solve(orc_solver *s, double tol, int32_t stop_rule, int64_t max_iter, int32_t check_every)
{
    if (check_every < 1) check_every = 1;
    for (;;) {
        if (s->have_metrics) {
            const double *M = s->metrics;
            int stop = stop_rule == 0 ? (M[M_RELKKT] <= tol)
                                      : (M[M_R] < (double)s->n * (double)s->m * tol);
            if (stop) return 1;
        }
        if (s->k >= max_iter) return 2;
        int check = ((s->k + 1) % check_every == 0) || (s->k + 1 >= max_iter);
        orc_step(s, check);
        if (!isfinite(s->metrics[M_DF]) || !isfinite(s->metrics[M_DY])) return 3;
    }
}

void orc_get_metrics(const orc_solver *s, double *out)
{
    memcpy(out, s->metrics, sizeof(double) * M_COUNT);
}

int32_t orc_metric_count(void) { return M_COUNT; }

double orc_get_eta(const orc_solver *s) { return s->eta; }

/* state = (F^{k-1/2}, Y^k, [k, omega, alpha, beta]) */
void orc_get_state(const orc_solver *s, double *F, double *Y, double *sc)
{
    if (F) memcpy(F, s->F, sizeof(double) * (size_t)s->n * s->m);
    if (Y) memcpy(Y, s->Y, sizeof(double) * (size_t)s->n * s->n);
    if (sc) {
        sc[0] = (double)s->k;
        sc[1] = s->omega;
        sc[2] = s->alpha;
        sc[3] = s->beta;
    }
}

void orc_set_state(orc_solver *s, const double *F, const double *Y, const double *sc)
{
    if (F) memcpy(s->F, F, sizeof(double) * (size_t)s->n * s->m);
    if (Y) memcpy(s->Y, Y, sizeof(double) * (size_t)s->n * s->n);
    if (sc) {
        s->k = (int64_t)sc[0];
        s->omega = sc[1];
        s->alpha = s->eta / s->omega;
        s->beta = s->eta * s->omega;
    }
    s->have_metrics = 0;
}

/* Fhat^{k-1/2} and T^ = -Fhat A^T of the last step (valid when it was checked),
 * plus Q of the last step for tests of the residual. */
void orc_get_last(const orc_solver *s, double *Fhat, double *That, double *Q)
{
    if (Fhat) memcpy(Fhat, s->Fhat, sizeof(double) * (size_t)s->n * s->m);
    if (That) memcpy(That, s->That, sizeof(double) * (size_t)s->n * s->n);
    if (Q) memcpy(Q, s->Q, sizeof(double) * (size_t)s->n * s->m);
}

/* test hook: write a NaN into F (which = 0) or Y (which = 1) at flat index idx */
void orc_poison(orc_solver *s, int32_t which, int64_t idx)
{
    if (which == 0 && idx >= 0 && idx < (int64_t)s->n * s->m) s->F[idx] = NAN;
    if (which == 1 && idx >= 0 && idx < (int64_t)s->n * s->n) s->Y[idx] = NAN;
}

/* the residual (e-res) and KKT quantities of an arbitrary (Q, Fhat = Pi(Q), Y)
 * triple, evaluated with this solver's problem data; results in metrics slots */
void orc_eval_residual(orc_solver *s, const double *Q, const double *Fhat, const double *Y, double *out)
{
    size_t nm = (size_t)s->n * s->m, nn = (size_t)s->n * s->n;
    memcpy(s->Q, Q, sizeof(double) * nm);
    memcpy(s->Fhat, Fhat, sizeof(double) * nm);
    double *Ysave = s->Y;
    double *Ytmp = (double *)malloc(sizeof(double) * nn);
    memcpy(Ytmp, Y, sizeof(double) * nn);
    s->Y = Ytmp;
    residual(s);
    s->Y = Ysave;
    free(Ytmp);
    memcpy(out, s->metrics, sizeof(double) * M_COUNT);
    s->have_metrics = 0;
}

int32_t orc_num_threads_available(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
