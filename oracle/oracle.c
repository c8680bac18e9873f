/* Test infrastructure -- the CPU oracle.  Only tests, the smoke check and the
 * benchmark's CPU-baseline leg load this library; the device library never
 * links, includes or calls it, and it shares no code with it.
 *
 * It computes, plainly and slowly, what the device path computes:
 *   - its own reader of the mechanism text;
 *   - the reactor right-hand side by definition (rhs_tmpl.h), in double and,
 *     for exact derivatives, in double complex (complex step: Squire & Trapp,
 *     SIAM Rev. 40 (1998));
 *   - a forward-difference Jacobian and a complex-step Jacobian, both dense;
 *   - dense LU with partial pivoting;
 *   - a 3-stage Radau IIA (order 5) integrator: collocation coefficients
 *     computed at start-up from the nodes (4-sqrt6)/10, (4+sqrt6)/10, 1,
 *     simplified Newton on the full 3n real stage system with the
 *     forward-difference Jacobian, error by step doubling, last step clipped
 *     to the requested interval (Hairer & Wanner, Solving ODEs II, Sec. IV.5
 *     and IV.8).  The converged stages solve the collocation equations, so an
 *     inexact Jacobian slows Newton down but does not change the result.
 *   - forward sensitivities s' = J s + (df/dtheta) d integrated beside y with
 *     the same Radau steps, directional derivatives by complex step.
 * Cells are independent (Sec. 1: each cell is its own reactor); OpenMP
 * threads take cells one at a time (the paper's chemistry load balancing,
 * Sec. 2.5, is what a dynamic schedule does on a CPU).
 */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OM_MAXSP 256
#define OM_MAXN (OM_MAXSP + 1)

/* reactor mode bits of the "mode" arguments below */
#define OM_ISOTHERMAL 1 /* T held fixed (f_T = 0) */
#define OM_CONSTV 2     /* constant volume: the p argument is the density */

enum { RX_PLAIN = 0, RX_THIRD = 1, RX_TROE = 2 };

typedef struct {
    int kind;
    double log10A, b, Ea;
    int nr, np;
    int sp_r[4], nu_r[4], sp_p[4], nu_p[4];
    double *alpha; /* [N] third-body efficiencies (1 unless listed) */
    double troe[7];
} omrxn;

typedef struct omech {
    int N, R_, E;
    double R, p0;
    char (*names)[32];
    double *W;    /* [N] kg/mol */
    int *comp;    /* [N*E] */
    double *nasa; /* [N*7] */
    omrxn *rx;
} omech;

/* ------------------------------------------------------------------------ */
/* mechanism reader                                                           */
/* ------------------------------------------------------------------------ */

static int find_species(const omech *m, const char *s)
{
    for (int k = 0; k < m->N; ++k)
        if (strcmp(m->names[k], s) == 0) return k;
    return -1;
}

void om_free(omech *m)
{
    if (!m) return;
    if (m->rx)
        for (int j = 0; j < m->R_; ++j) free(m->rx[j].alpha);
    free(m->rx);
    free(m->names);
    free(m->W);
    free(m->comp);
    free(m->nasa);
    free(m);
}

#define FAIL(...)                                 \
    do {                                          \
        snprintf(err, errlen, __VA_ARGS__);       \
        free(buf);                                \
        om_free(m);                               \
        return NULL;                              \
    } while (0)

omech *om_load(const char *text, char *err, int errlen)
{
    omech *m = calloc(1, sizeof(omech));
    char *buf = strdup(text);
    int nsp_read = 0, nth_read = 0, nrx_read = 0;
    omrxn *last = NULL;
    char *save = NULL;
    m->R = 8.314462618;
    m->p0 = 101325.0;
    for (char *line = strtok_r(buf, "\n", &save); line; line = strtok_r(NULL, "\n", &save)) {
        char *hash = strchr(line, '#');
        if (hash) *hash = 0;
        char *tok[64];
        int nt = 0;
        char *s2 = NULL;
        for (char *t = strtok_r(line, " \t\r", &s2); t && nt < 64; t = strtok_r(NULL, " \t\r", &s2))
            tok[nt++] = t;
        if (nt == 0) continue;
        if (!strcmp(tok[0], "STIFFCHEM-MECH") || !strcmp(tok[0], "NAME") || !strcmp(tok[0], "END")) continue;
        if (!strcmp(tok[0], "GAS_CONSTANT")) { m->R = atof(tok[1]); continue; }
        if (!strcmp(tok[0], "REF_PRESSURE")) { m->p0 = atof(tok[1]); continue; }
        if (!strcmp(tok[0], "ELEMENTS")) { m->E = atoi(tok[1]); continue; }
        if (!strcmp(tok[0], "SPECIES")) {
            m->N = atoi(tok[1]);
            if (m->N <= 0 || m->N > OM_MAXSP) FAIL("bad species count");
            m->names = calloc(m->N, 32);
            m->W = calloc(m->N, sizeof(double));
            m->comp = calloc((size_t)m->N * (m->E > 0 ? m->E : 1), sizeof(int));
            m->nasa = calloc((size_t)m->N * 7, sizeof(double));
            continue;
        }
        if (!strcmp(tok[0], "SP")) {
            if (nsp_read >= m->N || nt < 3 + m->E) FAIL("bad SP line");
            snprintf(m->names[nsp_read], 32, "%s", tok[1]);
            m->W[nsp_read] = atof(tok[2]);
            for (int e = 0; e < m->E; ++e) m->comp[nsp_read * m->E + e] = atoi(tok[3 + e]);
            ++nsp_read;
            continue;
        }
        if (!strcmp(tok[0], "NASA7")) {
            int k = find_species(m, tok[1]);
            if (k < 0 || nt < 9) FAIL("bad NASA7 line");
            for (int i = 0; i < 7; ++i) m->nasa[7 * k + i] = atof(tok[2 + i]);
            ++nth_read;
            continue;
        }
        if (!strcmp(tok[0], "REACTIONS")) {
            m->R_ = atoi(tok[1]);
            if (m->R_ <= 0) FAIL("bad reaction count");
            m->rx = calloc(m->R_, sizeof(omrxn));
            continue;
        }
        if (!strcmp(tok[0], "RX")) {
            if (nrx_read >= m->R_) FAIL("too many RX lines");
            omrxn *r = &m->rx[nrx_read++];
            r->kind = !strcmp(tok[1], "plain") ? RX_PLAIN : !strcmp(tok[1], "third") ? RX_THIRD
                      : !strcmp(tok[1], "troe") ? RX_TROE : -1;
            if (r->kind < 0) FAIL("bad reaction kind %s", tok[1]);
            r->log10A = atof(tok[2]);
            r->b = atof(tok[3]);
            r->Ea = atof(tok[4]);
            int p = 5;
            r->nr = atoi(tok[p++]);
            if (r->nr < 1 || r->nr > 4) FAIL("bad reactant count");
            for (int i = 0; i < r->nr; ++i) {
                r->sp_r[i] = find_species(m, tok[p++]);
                r->nu_r[i] = atoi(tok[p++]);
                if (r->sp_r[i] < 0) FAIL("unknown species");
            }
            r->np = atoi(tok[p++]);
            if (r->np < 1 || r->np > 4) FAIL("bad product count");
            for (int i = 0; i < r->np; ++i) {
                r->sp_p[i] = find_species(m, tok[p++]);
                r->nu_p[i] = atoi(tok[p++]);
                if (r->sp_p[i] < 0) FAIL("unknown species");
            }
            r->alpha = malloc(sizeof(double) * m->N);
            for (int k = 0; k < m->N; ++k) r->alpha[k] = 1.0;
            last = r;
            continue;
        }
        if (!strcmp(tok[0], "EFF")) {
            if (!last) FAIL("EFF without RX");
            int n = atoi(tok[1]);
            for (int i = 0; i < n; ++i) {
                int k = find_species(m, tok[2 + 2 * i]);
                if (k < 0) FAIL("unknown species in EFF");
                last->alpha[k] = atof(tok[3 + 2 * i]);
            }
            continue;
        }
        if (!strcmp(tok[0], "TROE")) {
            if (!last || nt < 8) FAIL("bad TROE line");
            for (int i = 0; i < 7; ++i) last->troe[i] = atof(tok[1 + i]);
            continue;
        }
        FAIL("unknown keyword %s", tok[0]);
    }
    if (nsp_read != m->N || nth_read != m->N || nrx_read != m->R_) FAIL("incomplete mechanism");
    free(buf);
    return m;
}

int om_n_species(const omech *m) { return m->N; }
int om_n_reactions(const omech *m) { return m->R_; }

/* ------------------------------------------------------------------------ */
/* right-hand side, real and complex                                          */
/* ------------------------------------------------------------------------ */

#define SC double
#define FN(x) x##_d
#define SEXP exp
#define SLOG log
#define SPOW(a, x) exp((x) * log(a))
#include "rhs_tmpl.h"
#undef SC
#undef FN
#undef SEXP
#undef SLOG
#undef SPOW

#define SC double complex
#define FN(x) x##_z
#define SEXP cexp
#define SLOG clog
#define SPOW(a, x) cexp((x) * log(a))
#include "rhs_tmpl.h"
#undef SC
#undef FN
#undef SEXP
#undef SLOG
#undef SPOW

void om_thermo(const omech *m, double T, double *cp_R, double *h_RT, double *s_R)
{
    for (int k = 0; k < m->N; ++k) thermo_d(m, k, T, &cp_R[k], &h_RT[k], &s_R[k]);
}

/* y = (Y_0..Y_{N-1}, T).  aux: rho, cp, sum h wdot, Wbar.  constv: p is rho. */
void om_rates(const omech *m, double p, const double *y, const double *dlnA, double *kf, double *kr,
              double *q, double *wdot, double *aux, int constv)
{
    rates_d(m, p, y, dlnA, kf, kr, q, wdot, aux, constv);
}

void om_rhs(const omech *m, double p, const double *y, const double *dlnA, double *f, int mode)
{
    rhs_d(m, p, y, dlnA, f, mode);
}

/* dense Jacobians, row-major J[i*(N+1)+j] = d f_i / d y_j */
void om_jac_fd(const omech *m, double p, const double *y, const double *dlnA, double *J, int mode)
{
    const int n = m->N + 1;
    double f0[OM_MAXN], f1[OM_MAXN], yp[OM_MAXN];
    rhs_d(m, p, y, dlnA, f0, mode);
    const double seps = sqrt(2.220446049250313e-16);
    for (int j = 0; j < n; ++j) {
        memcpy(yp, y, sizeof(double) * n);
        double typ = (j < m->N) ? 1e-10 : 1.0;
        double d = seps * fmax(fabs(y[j]), typ);
        yp[j] = y[j] + d;
        d = yp[j] - y[j];
        rhs_d(m, p, yp, dlnA, f1, mode);
        for (int i = 0; i < n; ++i) J[i * n + j] = (f1[i] - f0[i]) / d;
    }
}

static const double CS_H = 1e-30;

void om_jac_cs(const omech *m, double p, const double *y, const double *dlnA, double *J, int mode)
{
    const int n = m->N + 1;
    double complex yz[OM_MAXN], fz[OM_MAXN], dz[OM_MAXSP * 8];
    int R = m->R_;
    double complex *dl = NULL;
    if (dlnA) {
        dl = R <= OM_MAXSP * 8 ? dz : malloc(sizeof(double complex) * R);
        for (int j = 0; j < R; ++j) dl[j] = dlnA[j];
    }
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < n; ++i) yz[i] = y[i];
        yz[j] += I * CS_H;
        rhs_z(m, p, yz, dl, fz, mode);
        for (int i = 0; i < n; ++i) J[i * n + j] = cimag(fz[i]) / CS_H;
    }
    if (dl && dl != dz) free(dl);
}

/* F[i*R + j] = d f_i / d dlnA_j (complex step) */
void om_dfdp_cs(const omech *m, double p, const double *y, const double *dlnA, double *F)
{
    const int n = m->N + 1, R = m->R_;
    double complex yz[OM_MAXN], fz[OM_MAXN];
    double complex *dl = malloc(sizeof(double complex) * R);
    for (int i = 0; i < n; ++i) yz[i] = y[i];
    for (int j = 0; j < R; ++j) {
        for (int r = 0; r < R; ++r) dl[r] = dlnA ? dlnA[r] : 0.0;
        dl[j] += I * CS_H;
        rhs_z(m, p, yz, dl, fz, 0);
        for (int i = 0; i < n; ++i) F[i * R + j] = cimag(fz[i]) / CS_H;
    }
    free(dl);
}

/* ------------------------------------------------------------------------ */
/* dense LU with partial pivoting                                             */
/* ------------------------------------------------------------------------ */

int om_lu_factor(int n, double *A, int *piv)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(A[k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > best) { best = fabs(A[i * n + k]); p = i; }
        piv[k] = p;
        if (best == 0.0 || !isfinite(best)) return -1;
        if (p != k)
            for (int j = 0; j < n; ++j) { double t = A[k * n + j]; A[k * n + j] = A[p * n + j]; A[p * n + j] = t; }
        double inv = 1.0 / A[k * n + k];
        for (int i = k + 1; i < n; ++i) {
            double l = A[i * n + k] * inv;
            A[i * n + k] = l;
            if (l != 0.0)
                for (int j = k + 1; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
        }
    }
    return 0;
}

void om_lu_solve(int n, const double *LU, const int *piv, double *b)
{
    for (int k = 0; k < n; ++k)
        if (piv[k] != k) { double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < i; ++k) b[i] -= LU[i * n + k] * b[k];
    for (int i = n - 1; i >= 0; --i) {
        for (int k = i + 1; k < n; ++k) b[i] -= LU[i * n + k] * b[k];
        b[i] /= LU[i * n + i];
    }
}

/* solve A x = b (A, b overwritten; x returned in b); 0 on success */
int om_dense_solve(int n, double *A, double *b)
{
    int *piv = malloc(sizeof(int) * n);
    int rc = om_lu_factor(n, A, piv);
    if (rc == 0) om_lu_solve(n, A, piv, b);
    free(piv);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Radau IIA, 3 stages, order 5                                               */
/* ------------------------------------------------------------------------ */

static double RC[3], RA[9];

/* Collocation: c = roots of the Radau IIA polynomial on (0,1], A from the
 * simplifying assumption C(3): sum_j a_ij c_j^(q-1) = c_i^q / q, q = 1..3. */
static void radau_init(void)
{
    static int done = 0;
    if (done) return;
    double s6 = sqrt(6.0);
    RC[0] = (4.0 - s6) / 10.0;
    RC[1] = (4.0 + s6) / 10.0;
    RC[2] = 1.0;
    for (int i = 0; i < 3; ++i) {
        double V[9], rhs[3];
        for (int q = 0; q < 3; ++q) {
            for (int j = 0; j < 3; ++j) V[q * 3 + j] = pow(RC[j], q);
            rhs[q] = pow(RC[i], q + 1) / (q + 1);
        }
        om_dense_solve(3, V, rhs);
        for (int j = 0; j < 3; ++j) RA[i * 3 + j] = rhs[j];
    }
    done = 1;
}

void om_radau_coeffs(double *c, double *A)
{
    radau_init();
    memcpy(c, RC, sizeof RC);
    memcpy(A, RA, sizeof RA);
}

/* The integrated system: the reactor ODE, optionally augmented with ns
 * sensitivity vectors (forward-sensitivity mode).  z = (y, s_1..s_ns). */
typedef struct {
    const omech *m;
    double p;
    const double *dlnA;
    int mode;
    int ns;             /* number of sensitivity directions */
    const double *dpar; /* [ns][R] parameter directions (NULL: none) */
} sysdef;

static void sys_rhs(const sysdef *sd, const double *z, double *fz)
{
    const omech *m = sd->m;
    const int n = m->N + 1, R = m->R_;
    rhs_d(m, sd->p, z, sd->dlnA, fz, sd->mode);
    if (sd->ns == 0) return;
    double complex yz[OM_MAXN], out[OM_MAXN];
    double complex *dl = malloc(sizeof(double complex) * R);
    for (int s = 0; s < sd->ns; ++s) {
        const double *sv = z + n * (1 + s);
        for (int i = 0; i < n; ++i) yz[i] = z[i] + I * CS_H * sv[i];
        for (int j = 0; j < R; ++j)
            dl[j] = (sd->dlnA ? sd->dlnA[j] : 0.0) + (sd->dpar ? I * CS_H * sd->dpar[s * R + j] : 0.0);
        rhs_z(m, sd->p, yz, dl, out, sd->mode);
        for (int i = 0; i < n; ++i) fz[n * (1 + s) + i] = cimag(out[i]) / CS_H;
    }
    free(dl);
}

typedef struct {
    int n;  /* size of the state block */
    int nz; /* total size (n * (1+ns)) */
    double *J, *M, *F, *Z, *dZ, *yt, *ft;
    int *piv;
} radau_ws;

static double wrms(int n, const double *v, const double *sc)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) { double t = v[i] / sc[i]; s += t * t; }
    return sqrt(s / n);
}

/* One Radau step of size h from z (all blocks).  The Newton matrix is the
 * block-diagonal I - h A (x) J for every block (the coupling of the tangent
 * blocks to the state block is left out of the iteration matrix; the residual
 * is exact, so only the convergence rate is affected).  sc[nz] are the error
 * weights.  On success z1 = new state and 0 is returned; 1 if Newton failed. */
static int radau_step(const sysdef *sd, radau_ws *w, const double *z, double h, const double *sc,
                      double *z1)
{
    const int n = w->n, nz = w->nz, nb = nz / n, n3 = 3 * n;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int r = 0; r < n; ++r)
                for (int c = 0; c < n; ++c)
                    w->M[(i * n + r) * n3 + j * n + c] =
                        ((i == j && r == c) ? 1.0 : 0.0) - h * RA[i * 3 + j] * w->J[r * n + c];
    if (om_lu_factor(n3, w->M, w->piv) != 0) return 1;
    memset(w->Z, 0, sizeof(double) * 3 * nz);
    double prev = 0.0;
    for (int it = 0; it < 12; ++it) {
        for (int i = 0; i < 3; ++i) {
            for (int q = 0; q < nz; ++q) w->yt[q] = z[q] + w->Z[i * nz + q];
            sys_rhs(sd, w->yt, w->F + i * nz);
        }
        double nrm = 0.0;
        int bad = 0;
        for (int b = 0; b < nb; ++b) {
            double rhs[3 * OM_MAXN];
            for (int i = 0; i < 3; ++i)
                for (int r = 0; r < n; ++r) {
                    double acc = -w->Z[i * nz + b * n + r];
                    for (int j = 0; j < 3; ++j) acc += h * RA[i * 3 + j] * w->F[j * nz + b * n + r];
                    rhs[i * n + r] = acc;
                }
            om_lu_solve(n3, w->M, w->piv, rhs);
            for (int i = 0; i < 3; ++i)
                for (int r = 0; r < n; ++r) {
                    double d = rhs[i * n + r];
                    if (!isfinite(d)) bad = 1;
                    w->Z[i * nz + b * n + r] += d;
                    double t = d / sc[b * n + r];
                    nrm += t * t;
                }
        }
        if (bad) return 1;
        nrm = sqrt(nrm / (3.0 * nz));
        /* converged: increment a millionth of the local tolerance (the
         * roundoff floor at tight tolerances), or the contraction estimate
         * says the remaining error is below 1e-3 of it */
        int conv = nrm <= 1e-6;
        if (!conv && it >= 1) {
            double theta = nrm / prev;
            if (theta >= 0.99) return 1;
            conv = (theta / (1.0 - theta)) * nrm <= 1e-3;
        }
        if (conv) {
            for (int q = 0; q < nz; ++q) z1[q] = z[q] + w->Z[2 * nz + q];
            return 0;
        }
        prev = nrm;
    }
    return 1;
}

enum { CELL_OK = 0, CELL_MAX_STEPS = 1, CELL_H_UNDERFLOW = 2, CELL_NONFINITE = 3, CELL_BAD_INPUT = 4 };

/* Integrate one cell over [0, dt]: z in/out.  Error control on every
 * block.  Returns status; counts accepted/rejected doubled steps. */
static int radau_integrate(const sysdef *sd, double *z, double dt, double rtol, double atol, int max_steps,
                           int *nacc, int *nrej)
{
    const omech *m = sd->m;
    const int n = m->N + 1, nz = n * (1 + sd->ns);
    radau_init();
    radau_ws w;
    w.n = n;
    w.nz = nz;
    w.J = malloc(sizeof(double) * n * n);
    w.M = malloc(sizeof(double) * 9 * n * n);
    w.F = malloc(sizeof(double) * 3 * nz);
    w.Z = malloc(sizeof(double) * 3 * nz);
    w.yt = malloc(sizeof(double) * nz);
    w.piv = malloc(sizeof(int) * 3 * n);
    double *zh = malloc(sizeof(double) * nz), *zm = malloc(sizeof(double) * nz),
           *z2 = malloc(sizeof(double) * nz), *sc = malloc(sizeof(double) * nz), *err = malloc(sizeof(double) * nz);
    int status = CELL_OK;
    *nacc = *nrej = 0;
    double t = 0.0, h = 1e-3 * dt;
    int last_rejected = 0, nonfinite = 0;
    if (dt <= 0.0) goto done;
    while (t < dt) {
        if (*nacc + *nrej >= max_steps) { status = CELL_MAX_STEPS; break; }
        if (h < 1e-20 * dt) { status = CELL_H_UNDERFLOW; break; }
        int final = 0;
        if (t + h >= dt) { h = dt - t; final = 1; }
        om_jac_fd(m, sd->p, z, sd->dlnA, w.J, sd->mode);
        for (int i = 0; i < nz; ++i) sc[i] = atol + rtol * fabs(z[i]);
        int fail = radau_step(sd, &w, z, h, sc, zh);
        if (!fail) fail = radau_step(sd, &w, z, 0.5 * h, sc, zm);
        if (!fail) {
            om_jac_fd(m, sd->p, zm, sd->dlnA, w.J, sd->mode);
            fail = radau_step(sd, &w, zm, 0.5 * h, sc, z2);
        }
        if (fail) {
            ++*nrej;
            h *= 0.5;
            last_rejected = 1;
            continue;
        }
        for (int i = 0; i < nz; ++i) {
            sc[i] = atol + rtol * fmax(fabs(z[i]), fabs(z2[i]));
            err[i] = (z2[i] - zh[i]) / 31.0;
        }
        double e = wrms(nz, err, sc);
        if (!isfinite(e)) {
            ++*nrej;
            h *= 0.2;
            if (++nonfinite >= 5) { status = CELL_NONFINITE; break; }
            last_rejected = 1;
            continue;
        }
        nonfinite = 0;
        double fac = 0.9 * pow(fmax(e, 1e-300), -1.0 / 6.0);
        fac = fmin(6.0, fmax(0.2, fac));
        if (e <= 1.0) {
            ++*nacc;
            memcpy(z, z2, sizeof(double) * nz);
            t = final ? dt : t + h;
            if (last_rejected) fac = fmin(fac, 1.0);
            last_rejected = 0;
            h *= fac;
        } else {
            ++*nrej;
            last_rejected = 1;
            h *= fmin(fac, 1.0);
        }
    }
done:
    free(w.J); free(w.M); free(w.F); free(w.Z); free(w.yt); free(w.piv);
    free(zh); free(zm); free(z2); free(sc); free(err);
    return status;
}

/* Integrate ncells cells; Y0/Y1 are [ncells][N] (cell-major).  T1/Y1 may
 * alias T0/Y0.  dlnA: [R] or NULL.  Returns the number of failed cells. */
int om_integrate(const omech *m, int ncells, const double *T0, const double *p, const double *Y0,
                 const double *dt, const double *dlnA, double rtol, double atol, int max_steps,
                 double *T1, double *Y1, int *nacc, int *nrej, int *status, int nthreads, int mode)
{
    const int N = m->N;
    int nfail = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : nfail)
    for (int c = 0; c < ncells; ++c) {
        double z[OM_MAXN];
        for (int k = 0; k < N; ++k) z[k] = Y0[(size_t)c * N + k];
        z[N] = T0[c];
        int st = CELL_OK, na = 0, nr = 0;
        int ok = isfinite(z[N]) && z[N] > 0.0 && isfinite(p[c]) && p[c] > 0.0 && isfinite(dt[c]) && dt[c] >= 0.0;
        for (int k = 0; k < N; ++k) ok = ok && isfinite(z[k]);
        if (!ok) {
            st = CELL_BAD_INPUT;
        } else {
            sysdef sd = {m, p[c], dlnA, mode, 0, NULL};
            st = radau_integrate(&sd, z, dt[c], rtol, atol, max_steps, &na, &nr);
        }
        for (int k = 0; k < N; ++k) Y1[(size_t)c * N + k] = z[k];
        T1[c] = z[N];
        if (nacc) nacc[c] = na;
        if (nrej) nrej[c] = nr;
        if (status) status[c] = st;
        if (st != CELL_OK) ++nfail;
    }
    return nfail;
}

/* Forward sensitivities of one cell: integrate y and ns tangent vectors.
 * s0: [ns][N+1] initial tangents (d y0); dpar: [ns][R] parameter directions
 * in dlnA (NULL = none).  On return y (N+1) and s ([ns][N+1]) hold the final
 * state and tangents.  Returns the cell status. */
int om_integrate_sens(const omech *m, double p, double *y, double dt, const double *dlnA, int ns,
                      double *s, const double *dpar, double rtol, double atol, int max_steps, int *nacc,
                      int *nrej)
{
    const int n = m->N + 1;
    double *z = malloc(sizeof(double) * n * (1 + ns));
    memcpy(z, y, sizeof(double) * n);
    memcpy(z + n, s, sizeof(double) * n * ns);
    sysdef sd = {m, p, dlnA, 0, ns, dpar};
    int st = radau_integrate(&sd, z, dt, rtol, atol, max_steps, nacc, nrej);
    memcpy(y, z, sizeof(double) * n);
    memcpy(s, z + n, sizeof(double) * n * ns);
    free(z);
    return st;
}

/* Parallel driver for many (cell, direction-set) sensitivity problems. */
int om_integrate_sens_batch(const omech *m, int ncells, const double *p, double *y /*[nc][n]*/, const double *dt,
                            const double *dlnA, int ns, double *s /*[nc][ns][n]*/, const double *dpar /*[nc][ns][R] or NULL*/,
                            double rtol, double atol, int max_steps, int *status, int nthreads)
{
    const int n = m->N + 1, R = m->R_;
    int nfail = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : nfail)
    for (int c = 0; c < ncells; ++c) {
        int na, nr;
        int st = om_integrate_sens(m, p[c], y + (size_t)c * n, dt[c], dlnA, ns, s + (size_t)c * ns * n,
                                   dpar ? dpar + (size_t)c * ns * R : NULL, rtol, atol, max_steps, &na, &nr);
        status[c] = st;
        if (st) ++nfail;
    }
    return nfail;
}

int om_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
