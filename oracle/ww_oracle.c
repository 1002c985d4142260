/*
 * ww_oracle.c -- plain, slow, single-threaded CPU oracle for the MCF phase
 * unwrapping hot path of "A Probabilistic-Cost Algorithm for Large-Scale 2D
 * Phase Unwrapping" (Whirlwind).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke entry point and
 * the CPU-baseline leg of the benchmark may load this file.  It shares no code
 * with the HIP library and includes none of its headers.
 *
 * Everything is FP64 or integer.  Build with -O2 -ffp-contract=off.
 *
 * Conventions (m rows, n cols, row-major):
 *   x-edge hx(i,j) joins pixel (i,j) -> (i,j+1), i<m, j<n-1
 *   y-edge vy(i,j) joins pixel (i,j) -> (i+1,j), i<m-1, j<n
 *   loop p(i,j) has corners (i,j),(i,j+1),(i+1,j+1),(i+1,j), i<m-1, j<n-1
 *   dual node id of p(i,j) = i*(n-1)+j ; the ground node G = (m-1)*(n-1)
 *
 * Parity status of each function is recorded next to it ("pinned by ..." or
 * "parity unpinned").
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define WWO_OK 0
#define WWO_E_INVALID_ARG (-1)
#define WWO_E_OOM (-2)
#define WWO_E_INFEASIBLE (-3)
#define WWO_E_CERT (-6)

static const double PI_D = 3.14159265358979311599796346854;  /* double nearest pi */
static const double TWO_PI_D = 6.28318530717958623199592693709;

/* ------------------------------------------------------------------------ */
/* O0/O1  input normalisation, wrap counts, residues (Section II-A, eq. 1)  */
/* ------------------------------------------------------------------------ */

static double psi_eff(const float *psi, const uint8_t *valid, int64_t k) {
    if (valid && !valid[k]) return 0.0;
    return (double)psi[k];
}

/* integer number of 2pi cycles removed by wrap(): d = diff - 2pi*w in (-pi,pi] */
static int wrap_count(double diff) {
    if (diff > PI_D) return 1;
    if (diff <= -PI_D) return -1;
    return 0;
}

static int wx(const float *psi, const uint8_t *valid, int n, int i, int j) {
    int64_t a = (int64_t)i * n + j;
    return wrap_count(psi_eff(psi, valid, a + 1) - psi_eff(psi, valid, a));
}
static int wy(const float *psi, const uint8_t *valid, int n, int i, int j) {
    int64_t a = (int64_t)i * n + j;
    return wrap_count(psi_eff(psi, valid, a + n) - psi_eff(psi, valid, a));
}

/* Residue of every 2x2 loop (eq. 1, loop traversed (i,j)->(i,j+1)->(i+1,j+1)
 * ->(i+1,j)->(i,j)), the one-sided charges of the boundary ring (top, bottom,
 * left, right) and the ground charge, which balances the graph.
 * Pinned by exact rational recomputation, the vortex closed form and the
 * discrete Stokes identity. */
int wwo_residues(const float *psi, const uint8_t *valid, int m, int n,
                 int8_t *res, int8_t *perim, int64_t *ground) {
    if (m < 1 || n < 1) return WWO_E_INVALID_ARG;
    int64_t tot = 0;
    for (int i = 0; i + 1 < m; i++)
        for (int j = 0; j + 1 < n; j++) {
            int r = -(wx(psi, valid, n, i, j) + wy(psi, valid, n, i, j + 1)
                      - wx(psi, valid, n, i + 1, j) - wy(psi, valid, n, i, j));
            res[(int64_t)i * (n - 1) + j] = (int8_t)r;
            tot += r;
        }
    if (perim) {
        int64_t k = 0;
        for (int j = 0; j + 1 < n; j++) perim[k++] = (int8_t)(+wx(psi, valid, n, 0, j));
        for (int j = 0; j + 1 < n; j++) perim[k++] = (int8_t)(-wx(psi, valid, n, m - 1, j));
        for (int i = 0; i + 1 < m; i++) perim[k++] = (int8_t)(-wy(psi, valid, n, i, 0));
        for (int i = 0; i + 1 < m; i++) perim[k++] = (int8_t)(+wy(psi, valid, n, i, n - 1));
    }
    if (ground) *ground = -tot;
    return WWO_OK;
}

/* ------------------------------------------------------------------------ */
/* O3  cost table (Section II-B, eqs. 4-7)                                   */
/* ------------------------------------------------------------------------ */

/* Positive-term hypergeometric sum F(z) = 2F1(2, 2L; L+3/2; z), 0 <= z <= 1/2,
 * summed until a term is below 2^-60 of the partial sum after the terms have
 * started to decrease. */
static double hyp_2_2L(int L, double z) {
    double s = 0.0, t = 1.0;
    for (int k = 0; k < 100000; k++) {
        s += t;
        double r = (2.0 + k) * (2.0 * L + k) / ((L + 1.5 + k) * (k + 1.0)) * z;
        t *= r;
        if (r < 1.0 && t < s * 8.673617379884035e-19) break;
    }
    return s;
}

/* Multilook phase-noise density f_eta(eta | gamma, L) of Lee et al. (1994),
 * the density named in Section II-B.  With beta = gamma cos(eta) it equals
 *   (1-g^2)^L / (2 pi (2L+1)) * 2F1(2, 2L; L+3/2; (1+beta)/2),
 * a sum of positive terms, used for beta <= 0; for beta > 0 the identity
 * f(beta) = f(-beta) + 2 T1(beta), where T1 is the odd (first) term of the
 * published two-term form, keeps both parts positive.  Pinned against the
 * published form at 300 digits, the L=1 closed form, normalisation and the
 * uniform limit at gamma = 0. */
/* log(1 - x^2) = log1p(-x) + log1p(x), accurate for x near 1 */
static double log_one_minus_sq(double x) { return log1p(-x) + log1p(x); }

double wwo_f_eta(double eta, double g, int L) {
    double b = g * cos(eta);
    double lg = log_one_minus_sq(g);
    double pref = exp((double)L * lg) / (2.0 * PI_D * (2.0 * L + 1.0));
    if (b <= 0.0) return pref * hyp_2_2L(L, 0.5 * (1.0 + b));
    double s = pref * hyp_2_2L(L, 0.5 * (1.0 - b));
    double lb = log_one_minus_sq(b);
    double lr = lgamma(L + 0.5) - lgamma((double)L);
    double t1 = exp(lr + (double)L * (lg - lb) - 0.5 * lb) * b / (2.0 * sqrt(PI_D));
    return s + 2.0 * t1;
}

/* Density of the sample coherence estimate (eq. 3) given the true coherence,
 * Touzi et al. (1999), Section II-B eq. 5:
 *   2(L-1)(1-g^2)^L gh (1-gh^2)^(L-2) 2F1(L, L; 1; g^2 gh^2)
 * with 2F1(L,L;1;x) = (1-x)^(1-2L) sum_k C(L-1,k)^2 x^k (Euler transform).
 * Pinned by normalisation in gh and the finite form against mpmath. */
double wwo_touzi(double gh, double g, int L) {
    if (L < 2 || gh <= 0.0 || gh >= 1.0) return 0.0;
    double x = g * g * gh * gh;
    double lp = log(2.0 * (L - 1)) + (double)L * log_one_minus_sq(g) + log(gh)
                + (double)(L - 2) * log_one_minus_sq(gh) + (double)(1 - 2 * L) * log1p(-x);
    double c = 1.0, poly = 0.0, xp = 1.0;
    for (int k = 0; k <= L - 1; k++) {
        poly += c * c * xp;
        xp *= x;
        c = c * (double)(L - 1 - k) / (double)(k + 1);
    }
    return exp(lp) * poly;
}

/* Gauss-Legendre nodes/weights on [-1, 1] (Newton iteration on P_n). */
void wwo_gauss_legendre(int n, double *x, double *w) {
    for (int i = 0; i < n; i++) {
        double z = cos(PI_D * (i + 0.75) / (n + 0.5));
        double pp = 0.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            pp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / pp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        /* recompute derivative at the converged node */
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; k++) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        pp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = -z;  /* ascending */
        w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

typedef struct {
    int32_t n_alpha, n_gamma, n_eta, n_gpanel, n_gnode, n_aquad;
    double sigma_span;
} wwo_lut_params;

static void default_lut_params(wwo_lut_params *p) {
    p->n_alpha = 128; p->n_gamma = 64; p->n_eta = 2048;
    p->n_gpanel = 64; p->n_gnode = 16; p->n_aquad = 513; p->sigma_span = 8.0;
}

/* Composite Gauss-Legendre rule on [0,1] for the true coherence: n_gpanel
 * equal panels of n_gnode nodes each (ascending). */
static int gamma_rule(const wwo_lut_params *p, double **gx_out, double **gw_out) {
    int Q = p->n_gnode, P = p->n_gpanel;
    double *x = malloc(sizeof(double) * Q), *w = malloc(sizeof(double) * Q);
    double *gx = malloc(sizeof(double) * P * Q), *gw = malloc(sizeof(double) * P * Q);
    if (!x || !w || !gx || !gw) { free(x); free(w); free(gx); free(gw); return WWO_E_OOM; }
    wwo_gauss_legendre(Q, x, w);
    for (int pa = 0; pa < P; pa++)
        for (int q = 0; q < Q; q++) {
            gx[pa * Q + q] = (pa + 0.5 * (1.0 + x[q])) / P;
            gw[pa * Q + q] = w[q] / (2.0 * P);
        }
    free(x); free(w);
    *gx_out = gx; *gw_out = gw;
    return WWO_OK;
}

/* f~ from a precomputed table fe[k*N + i] = f_eta(eta_i | gamma_k, L). */
static void ftilde_from_table(int L, double gh, int N, int NQ, const double *gx, const double *gw,
                              const double *fe, double *out) {
    double deta = TWO_PI_D / N;
    for (int i = 0; i < N; i++) out[i] = 0.0;
    for (int k = 0; k < NQ; k++) {
        double W = gw[k] * wwo_touzi(gh, gx[k], L);
        if (W == 0.0) continue;
        for (int i = 0; i < N; i++) out[i] += W * fe[(int64_t)k * N + i];
    }
    double mass = 0.0;
    for (int i = 0; i < N; i++) mass += out[i] * deta;
    for (int i = 0; i < N; i++) out[i] /= mass;
}

static double *f_eta_table(int L, int N, int NQ, const double *gx) {
    double *fe = malloc(sizeof(double) * (size_t)NQ * N);
    if (!fe) return NULL;
    double deta = TWO_PI_D / N;
    for (int k = 0; k < NQ; k++)
        for (int i = 0; i < N; i++)
            fe[(int64_t)k * N + i] = wwo_f_eta(-PI_D + (i + 0.5) * deta, gx[k], L);
    return fe;
}

/* Coherence-marginalised phase density (eq. 5) for one sample coherence gh, on
 * the eta midpoints eta_i = -pi + (i + 1/2) 2pi/N, normalised to unit mass
 * (eq. 5 is stated up to proportionality).  The integral over the true
 * coherence uses the composite Gauss-Legendre rule above.  Pinned by
 * normalisation and adaptive quadrature of the same integral. */
int wwo_ftilde(int L, double gh, const wwo_lut_params *pin, double *out) {
    wwo_lut_params p;
    if (pin) p = *pin; else default_lut_params(&p);
    double *gx, *gw;
    if (gamma_rule(&p, &gx, &gw)) return WWO_E_OOM;
    int NQ = p.n_gpanel * p.n_gnode;
    double *fe = f_eta_table(L, p.n_eta, NQ, gx);
    if (!fe) { free(gx); free(gw); return WWO_E_OOM; }
    ftilde_from_table(L, gh, p.n_eta, NQ, gx, gw, fe, out);
    free(fe); free(gx); free(gw);
    return WWO_OK;
}

/* Edge-noise masses (difference of two independent phase errors, the
 * self-convolution of f~, Section II-B): pm[s + N-1] = deta^2 sum_i
 * f~[i+s] f~[i] for s = -(N-1)..(N-1); the mass of cell s is spread uniformly
 * over [(s-1/2) deta, (s+1/2) deta]. */
void wwo_edge_mass(const double *ft, int N, double *pm) {
    double deta = TWO_PI_D / N;
    for (int s = -(N - 1); s <= N - 1; s++) {
        double acc = 0.0;
        for (int i = 0; i < N; i++) {
            int k = i + s;
            if (k < 0 || k >= N) continue;
            acc += ft[k] * ft[i];
        }
        pm[s + N - 1] = acc * deta * deta;
    }
}

typedef struct {
    int N;
    double deta;
    const double *pm;   /* 2N-1 cell masses */
    double *CL, *CR;    /* 2N entries each, index k + N-1 for edge k = -(N-1)..N */
} edge_cdf;

static void cdf_build(edge_cdf *c) {
    int N = c->N;
    c->CL[0] = 0.0;
    for (int k = -(N - 1) + 1; k <= N; k++) c->CL[k + N - 1] = c->CL[k - 1 + N - 1] + c->pm[k - 1 + N - 1];
    c->CR[2 * N - 1] = 0.0;
    for (int k = N - 1; k >= -(N - 1); k--) c->CR[k + N - 1] = c->CR[k + 1 + N - 1] + c->pm[k + N - 1];
}

/* mass below x (left cumulative, linear inside a cell) */
static double G_left(const edge_cdf *c, double x) {
    int N = c->N;
    double u = x / c->deta + 0.5;
    double fk = floor(u);
    if (fk < -(N - 1)) return 0.0;
    if (fk > N - 1) return c->CL[2 * N - 1];
    int k = (int)fk;
    double t = u - fk;
    return c->CL[k + N - 1] + t * c->pm[k + N - 1];
}
/* mass above x (right cumulative, summed from the far end) */
static double G_right(const edge_cdf *c, double x) {
    int N = c->N;
    double u = x / c->deta + 0.5;
    double fk = floor(u);
    if (fk < -(N - 1)) return c->CR[0];
    if (fk > N - 1) return 0.0;
    int k = (int)fk;
    double t = u - fk;
    return c->CR[k + 1 + N - 1] + (1.0 - t) * c->pm[k + N - 1];
}

/* Branch probabilities of eq. 6 for true slope alpha. */
static void branch_q(const edge_cdf *c, double alpha, double *q0, double *qp) {
    if (alpha <= 0.0) *q0 = G_right(c, -PI_D - alpha) - G_right(c, PI_D - alpha);
    else *q0 = G_left(c, PI_D - alpha) - G_left(c, -PI_D - alpha);
    *qp = G_right(c, PI_D - alpha);
}

int wwo_branch_q(const double *pm, int N, double alpha, double *q0, double *qp) {
    edge_cdf c;
    c.N = N; c.deta = TWO_PI_D / N; c.pm = pm;
    c.CL = malloc(sizeof(double) * 2 * N);
    c.CR = malloc(sizeof(double) * 2 * N);
    if (!c.CL || !c.CR) { free(c.CL); free(c.CR); return WWO_E_OOM; }
    cdf_build(&c);
    branch_q(&c, alpha, q0, qp);
    free(c.CL); free(c.CR);
    return WWO_OK;
}

/* Slope-error standard deviation sigma_alpha(gh): the standard deviation of
 * the single-pixel phase noise at gamma = gh, which equals pi/sqrt(3) at zero
 * coherence as Section II-B requires.  Fidelity to the paper's own formula is
 * unpinned (the reading is recorded in the design notes). */
double wwo_sigma_alpha(double gh, int L, int N) {
    double deta = TWO_PI_D / N, acc = 0.0;
    for (int i = 0; i < N; i++) {
        double eta = -PI_D + (i + 0.5) * deta;
        acc += eta * eta * wwo_f_eta(eta, gh, L) * deta;
    }
    return sqrt(acc);
}

/* Slope marginalisation (eq. 7): P_j = sum_k om_k q_j(alpha_k) over NQ uniform
 * nodes alpha_k = ah + span*sig*(2k/(NQ-1) - 1) with normalised Gaussian
 * weights om (flat prior on the true slope). */
static void slope_marginal(const edge_cdf *c, double ah, double sig, int NQ, double span,
                           const double *om, double *P0o, double *Ppo) {
    double P0 = 0.0, Pp = 0.0;
    for (int k = 0; k < NQ; k++) {
        double a = ah + span * sig * (2.0 * k / (NQ - 1) - 1.0);
        double q0, qp;
        branch_q(c, a, &q0, &qp);
        P0 += om[k] * q0;
        Pp += om[k] * qp;
    }
    *P0o = P0;
    *Ppo = Pp;
}

static void gauss_weights(int NQ, double span, double *om) {
    double osum = 0.0;
    for (int k = 0; k < NQ; k++) {
        double u = span * (2.0 * k / (NQ - 1) - 1.0);
        om[k] = exp(-0.5 * u * u);
        osum += om[k];
    }
    for (int k = 0; k < NQ; k++) om[k] /= osum;
}

int wwo_slope_marginal(const double *pm, int N, double ah, double sig, int NQ, double span,
                       double *P0, double *Pp) {
    edge_cdf c;
    c.N = N; c.deta = TWO_PI_D / N; c.pm = pm;
    c.CL = malloc(sizeof(double) * 2 * N);
    c.CR = malloc(sizeof(double) * 2 * N);
    double *om = malloc(sizeof(double) * NQ);
    if (!c.CL || !c.CR || !om) { free(c.CL); free(c.CR); free(om); return WWO_E_OOM; }
    cdf_build(&c);
    gauss_weights(NQ, span, om);
    slope_marginal(&c, ah, sig, NQ, span, om, P0, Pp);
    free(c.CL); free(c.CR); free(om);
    return WWO_OK;
}

/* Cost table T[c][b] = min(32767, floor(100 max{0, -ln(P+/P0)})) at bin
 * centres alpha_b = -pi + (b+1/2) 2pi/N_alpha, gh_c = (c+1/2)/N_gamma (eqs.
 * 4-7).  P0/Pp/sig may be NULL.  Returns WWO_OK. */
int wwo_build_lut(int L, const wwo_lut_params *pin, int16_t *T, double *P0o, double *Ppo,
                  double *sigo) {
    if (L < 2 || L > 64) return WWO_E_INVALID_ARG;
    wwo_lut_params p;
    if (pin) p = *pin; else default_lut_params(&p);
    int N = p.n_eta, NA = p.n_alpha, NG = p.n_gamma, NQ = p.n_aquad;
    double *ft = malloc(sizeof(double) * N);
    double *pm = malloc(sizeof(double) * (2 * N - 1));
    double *om = malloc(sizeof(double) * NQ);
    edge_cdf c;
    c.N = N; c.deta = TWO_PI_D / N; c.pm = pm;
    c.CL = malloc(sizeof(double) * 2 * N);
    c.CR = malloc(sizeof(double) * 2 * N);
    if (!ft || !pm || !om || !c.CL || !c.CR) {
        free(ft); free(pm); free(om); free(c.CL); free(c.CR);
        return WWO_E_OOM;
    }
    /* normalised Gaussian weights over alpha_hat +- span*sigma (eq. 7) */
    double *gx, *gw;
    if (gamma_rule(&p, &gx, &gw)) { free(ft); free(pm); free(om); free(c.CL); free(c.CR); return WWO_E_OOM; }
    int NGQ = p.n_gpanel * p.n_gnode;
    double *fe = f_eta_table(L, N, NGQ, gx);
    if (!fe) { free(gx); free(gw); free(ft); free(pm); free(om); free(c.CL); free(c.CR); return WWO_E_OOM; }
    gauss_weights(NQ, p.sigma_span, om);

    for (int cg = 0; cg < NG; cg++) {
        double gh = (cg + 0.5) / NG;
        ftilde_from_table(L, gh, N, NGQ, gx, gw, fe, ft);
        wwo_edge_mass(ft, N, pm);
        cdf_build(&c);
        double sig = wwo_sigma_alpha(gh, L, N);
        if (sigo) sigo[cg] = sig;
        for (int b = 0; b < NA; b++) {
            double ah = -PI_D + (b + 0.5) * TWO_PI_D / NA;
            double P0, Pp;
            slope_marginal(&c, ah, sig, NQ, p.sigma_span, om, &P0, &Pp);
            int16_t t;
            if (!(Pp > 0.0)) t = 32767;
            else {
                double cst = -log(Pp / P0);
                if (cst < 0.0) cst = 0.0;
                double v = floor(100.0 * cst);
                t = v >= 32767.0 ? (int16_t)32767 : (int16_t)v;
            }
            T[(int64_t)cg * NA + b] = t;
            if (P0o) P0o[(int64_t)cg * NA + b] = P0;
            if (Ppo) Ppo[(int64_t)cg * NA + b] = Pp;
        }
    }
    free(fe); free(gx); free(gw);
    free(ft); free(pm); free(om); free(c.CL); free(c.CR);
    return WWO_OK;
}

/* The table at a non-integer number of looks (Section II-B: the table is
 * precomputed on a grid that includes L and read by interpolation at run
 * time).  The L grid is the integers; an effective L given in 2^-16 fixed
 * point, L = l0 + f / 2^16 with 0 <= f < 2^16, blends the tables of the
 * two neighbouring integers entry by entry:
 *   T[c][b] = floor((T_l0[c][b] (2^16 - f) + T_l0+1[c][b] f) / 2^16),
 * so f = 0 gives T_l0 itself.  n entries.  Pinned by the integer nodes,
 * the halfway floor-of-mean, and agreement with numpy's linear
 * interpolation over L and with the model evaluated at non-integer L. */
void wwo_lut_blend_looks(const int16_t *T0, const int16_t *T1, int64_t n, int32_t f, int16_t *out) {
    for (int64_t k = 0; k < n; k++)
        out[k] = (int16_t)(((int64_t)T0[k] * (65536 - f) + (int64_t)T1[k] * f) >> 16);
}

/* ------------------------------------------------------------------------ */
/* O4  per-edge integer costs (Section II-B: slope box filter, edge          */
/*     coherence = min of endpoints, LUT lookup, mirror, mask, steep rule)   */
/* ------------------------------------------------------------------------ */

static const int64_t PFIX = 3294199;  /* round(pi * 2^20) */

typedef struct { double key; int64_t id; } steep_cand;

static int steep_cmp(const void *a, const void *b) {
    const steep_cand *x = a, *y = b;
    if (x->key > y->key) return -1;
    if (x->key < y->key) return 1;
    return (x->id < y->id) ? -1 : (x->id > y->id);
}

static double coh_eff(const float *coh, int64_t k) {
    double c = (double)coh[k];
    if (!(c > 0.0)) return 0.0;  /* also NaN */
    if (c > 1.0) return 1.0;
    return c;
}

/* The cost pair (c+, c-) of an edge from the table T[N_gamma][N_alpha].
 * The slope position of the box mean is s = (S + K P) N_alpha / (2 K P)
 * (bin b spans [b, b+1)); the coherence position is g N_gamma.
 * interp == 0 (nearest bin, Section II-B read as the table's own bins):
 *   c+ = T[floor(g N_gamma)][floor(s)], c- = T[..][N_alpha - 1 - floor(s)].
 * interp == 1 (the table interpolated at run time, Section II-B): positions
 *   relative to the bin centres, t = s - 1/2 and u = g N_gamma - 1/2, in
 *   2^-16 fixed point (t16 = floor(s 2^16) - 2^15, likewise u16), split into
 *   a cell index and a fraction, clamped to the outermost centres; the
 *   bilinear blend of the four surrounding entries is rounded down.  c-
 *   uses the mirrored position (N_alpha - 1) 2^16 - t16. */
static int16_t lut_blend(const int16_t *T, int NA, int NG, int64_t t16, int64_t u16) {
    int64_t ia = t16 >> 16, fa = t16 - (ia << 16);
    int64_t ig = u16 >> 16, fg = u16 - (ig << 16);
    if (ia < 0) { ia = 0; fa = 0; }
    if (ia >= NA - 1) { ia = NA - 1; fa = 0; }
    if (ig < 0) { ig = 0; fg = 0; }
    if (ig >= NG - 1) { ig = NG - 1; fg = 0; }
    const int64_t ib = ia + 1 < NA ? ia + 1 : ia, jg = ig + 1 < NG ? ig + 1 : ig;
    const int64_t r0 = (int64_t)T[ig * NA + ia] * (65536 - fa) + (int64_t)T[ig * NA + ib] * fa;
    const int64_t r1 = (int64_t)T[jg * NA + ia] * (65536 - fa) + (int64_t)T[jg * NA + ib] * fa;
    return (int16_t)((r0 * (65536 - fg) + r1 * fg) >> 32);
}

void wwo_lut_pair(const int16_t *T, int NA, int NG, int64_t S, int64_t K, double g, int interp,
                  int16_t *cp, int16_t *cn) {
    const int64_t num = (S + K * PFIX) * NA, den = 2 * K * PFIX;
    if (!interp) {
        int64_t ba = num / den;
        if (ba < 0) ba = 0;
        if (ba > NA - 1) ba = NA - 1;
        int64_t bg = (int64_t)floor(g * NG);
        if (bg > NG - 1) bg = NG - 1;
        *cp = T[bg * NA + ba];
        *cn = T[bg * NA + (NA - 1 - ba)];
        return;
    }
    const int64_t t16 = (num * 65536) / den - 32768;
    const int64_t u16 = (int64_t)floor(g * NG * 65536.0) - 32768;
    *cp = lut_blend(T, NA, NG, t16, u16);
    *cn = lut_blend(T, NA, NG, (int64_t)(NA - 1) * 65536 - t16, u16);
}

/* Edge costs c+ (the arc that raises the edge's cycle difference by one) and
 * c- (lowers it): c+ = T[bg][ba], c- = T[bg][N_alpha-1-ba].  ba is the bin of
 * the box-filtered (side 2h+1, clipped, valid samples only) wrapped gradient in
 * 2^-20 rad fixed point; bg the bin of min(coh_u, coh_v).  Edges with an
 * invalid endpoint cost 0.  Steep rule: valid edges with |d| > thresh get cost
 * 0, at most floor(cap_pct * valid_edges / 100) of them, largest |d| first,
 * ties by edge id (x-edges row-major, then y-edges row-major).
 * interp selects the table lookup of wwo_lut_pair.
 * stats (nullable): [0]=valid edges, [1]=steep candidates, [2]=zeroed.
 * Pinned by mirror symmetry, mask, steep count and an independent numpy
 * recomputation. */
int wwo_edge_costs(const float *psi, const float *coh, const uint8_t *valid, int m, int n,
                   const int16_t *T, int n_alpha, int n_gamma, int box_half,
                   int steep_rule, double steep_thresh, int steep_cap_pct, int interp,
                   int16_t *cxp, int16_t *cxn, int16_t *cyp, int16_t *cyn, int64_t *stats) {
    if (m < 1 || n < 1 || box_half < 0) return WWO_E_INVALID_ARG;
    int64_t nx = (int64_t)m * (n - 1), ny = (int64_t)(m - 1) * n;
    if (n < 2) nx = 0;
    if (m < 2) ny = 0;
    int32_t *qx = malloc(sizeof(int32_t) * (nx ? nx : 1));
    int32_t *qy = malloc(sizeof(int32_t) * (ny ? ny : 1));
    uint8_t *vx = malloc(nx ? nx : 1), *vy = malloc(ny ? ny : 1);
    double *dx = malloc(sizeof(double) * (nx ? nx : 1));
    double *dy = malloc(sizeof(double) * (ny ? ny : 1));
    if (!qx || !qy || !vx || !vy || !dx || !dy) {
        free(qx); free(qy); free(vx); free(vy); free(dx); free(dy);
        return WWO_E_OOM;
    }
    /* wrapped gradients, fixed point, validity */
    for (int i = 0; i < m; i++)
        for (int j = 0; j + 1 < n; j++) {
            int64_t a = (int64_t)i * n + j, e = (int64_t)i * (n - 1) + j;
            double diff = psi_eff(psi, valid, a + 1) - psi_eff(psi, valid, a);
            double d = diff - TWO_PI_D * wrap_count(diff);
            dx[e] = d;
            qx[e] = (int32_t)floor(d * 1048576.0);
            vx[e] = (!valid) || (valid[a] && valid[a + 1]);
        }
    for (int i = 0; i + 1 < m; i++)
        for (int j = 0; j < n; j++) {
            int64_t a = (int64_t)i * n + j, e = (int64_t)i * n + j;
            double diff = psi_eff(psi, valid, a + n) - psi_eff(psi, valid, a);
            double d = diff - TWO_PI_D * wrap_count(diff);
            dy[e] = d;
            qy[e] = (int32_t)floor(d * 1048576.0);
            vy[e] = (!valid) || (valid[a] && valid[a + n]);
        }
    int h = box_half;
    /* x-edges: array m x (n-1) */
    for (int i = 0; i < m; i++)
        for (int j = 0; j + 1 < n; j++) {
            int64_t e = (int64_t)i * (n - 1) + j;
            if (!vx[e]) { cxp[e] = 0; cxn[e] = 0; continue; }
            int64_t S = 0, cnt = 0;
            for (int ii = i - h; ii <= i + h; ii++) {
                if (ii < 0 || ii >= m) continue;
                for (int jj = j - h; jj <= j + h; jj++) {
                    if (jj < 0 || jj >= n - 1) continue;
                    int64_t f = (int64_t)ii * (n - 1) + jj;
                    if (!vx[f]) continue;
                    S += qx[f];
                    cnt++;
                }
            }
            int64_t a = (int64_t)i * n + j;
            double g = fmin(coh_eff(coh, a), coh_eff(coh, a + 1));
            wwo_lut_pair(T, n_alpha, n_gamma, S, cnt, g, interp, &cxp[e], &cxn[e]);
        }
    /* y-edges: array (m-1) x n */
    for (int i = 0; i + 1 < m; i++)
        for (int j = 0; j < n; j++) {
            int64_t e = (int64_t)i * n + j;
            if (!vy[e]) { cyp[e] = 0; cyn[e] = 0; continue; }
            int64_t S = 0, cnt = 0;
            for (int ii = i - h; ii <= i + h; ii++) {
                if (ii < 0 || ii >= m - 1) continue;
                for (int jj = j - h; jj <= j + h; jj++) {
                    if (jj < 0 || jj >= n) continue;
                    int64_t f = (int64_t)ii * n + jj;
                    if (!vy[f]) continue;
                    S += qy[f];
                    cnt++;
                }
            }
            int64_t a = (int64_t)i * n + j;
            double g = fmin(coh_eff(coh, a), coh_eff(coh, a + n));
            wwo_lut_pair(T, n_alpha, n_gamma, S, cnt, g, interp, &cyp[e], &cyn[e]);
        }
    /* steep-gradient rule */
    int64_t nvalid = 0, ncand = 0, nzero = 0;
    for (int64_t e = 0; e < nx; e++) nvalid += vx[e];
    for (int64_t e = 0; e < ny; e++) nvalid += vy[e];
    if (steep_rule) {
        for (int64_t e = 0; e < nx; e++) ncand += vx[e] && fabs(dx[e]) > steep_thresh;
        for (int64_t e = 0; e < ny; e++) ncand += vy[e] && fabs(dy[e]) > steep_thresh;
        int64_t cap = (nvalid * steep_cap_pct) / 100;
        steep_cand *cs = malloc(sizeof(steep_cand) * (ncand ? ncand : 1));
        if (!cs) { free(qx); free(qy); free(vx); free(vy); free(dx); free(dy); return WWO_E_OOM; }
        int64_t k = 0;
        for (int64_t e = 0; e < nx; e++)
            if (vx[e] && fabs(dx[e]) > steep_thresh) { cs[k].key = fabs(dx[e]); cs[k].id = e; k++; }
        for (int64_t e = 0; e < ny; e++)
            if (vy[e] && fabs(dy[e]) > steep_thresh) { cs[k].key = fabs(dy[e]); cs[k].id = nx + e; k++; }
        if (ncand > cap) qsort(cs, ncand, sizeof(steep_cand), steep_cmp);
        nzero = ncand > cap ? cap : ncand;
        for (int64_t t = 0; t < nzero; t++) {
            int64_t id = cs[t].id;
            if (id < nx) { cxp[id] = 0; cxn[id] = 0; }
            else { cyp[id - nx] = 0; cyn[id - nx] = 0; }
        }
        free(cs);
    }
    if (stats) { stats[0] = nvalid; stats[1] = ncand; stats[2] = nzero; }
    free(qx); free(qy); free(vx); free(vy); free(dx); free(dy);
    return WWO_OK;
}

/* ------------------------------------------------------------------------ */
/* O5  min-cost flow by successive shortest paths (Section II-A eq. 2,      */
/*     Section II-C): one path at a time, binary heap, node potentials.      */
/* ------------------------------------------------------------------------ */

/* A residual move of +1 or -1 on an edge whose net flow (cycle difference)
 * is f.  Returns 0 and sets *cost when the move is allowed. */
static int move_cost(int f, int delta, int cp, int cn, int64_t *cost) {
    if (f == 0) { *cost = delta > 0 ? cp : cn; return 0; }
    if (f == -delta) { *cost = -(int64_t)(f > 0 ? cp : cn); return 0; }
    return -1;
}

typedef struct {
    int m, n, R, C;          /* R = m-1 loop rows, C = n-1 loop cols */
    int64_t nn, G;           /* nodes incl. ground, ground id */
    const int16_t *cxp, *cxn, *cyp, *cyn;
    int8_t *fx, *fy;         /* net flow (cycle difference) per edge */
} graph;

/* Enumerate the arcs leaving node u.  For each: head node, edge kind (0 = x,
 * 1 = y), edge index and the move (+1/-1) applied to that edge's net flow. */
typedef struct { int64_t v; int kind; int64_t e; int delta; } arc;

static int out_arcs(const graph *g, int64_t u, arc *out) {
    int k = 0;
    int R = g->R, C = g->C, n = g->n, m = g->m;
    if (u != g->G) {
        int i = (int)(u / C), j = (int)(u % C);
        /* up across hx(i,j): cycle difference -1 */
        out[k].v = (i > 0) ? u - C : g->G; out[k].kind = 0; out[k].e = (int64_t)i * (n - 1) + j; out[k].delta = -1; k++;
        /* down across hx(i+1,j): +1 */
        out[k].v = (i + 1 < R) ? u + C : g->G; out[k].kind = 0; out[k].e = (int64_t)(i + 1) * (n - 1) + j; out[k].delta = +1; k++;
        /* left across vy(i,j): +1 */
        out[k].v = (j > 0) ? u - 1 : g->G; out[k].kind = 1; out[k].e = (int64_t)i * n + j; out[k].delta = +1; k++;
        /* right across vy(i,j+1): -1 */
        out[k].v = (j + 1 < C) ? u + 1 : g->G; out[k].kind = 1; out[k].e = (int64_t)i * n + j + 1; out[k].delta = -1; k++;
        return k;
    }
    /* ground: one arc into every perimeter loop */
    for (int j = 0; j < C; j++) {  /* top edges hx(0,j): ground -> p(0,j) is downward: +1 */
        out[k].v = j; out[k].kind = 0; out[k].e = j; out[k].delta = +1; k++;
    }
    for (int j = 0; j < C; j++) {  /* bottom edges hx(m-1,j): ground -> p(R-1,j) upward: -1 */
        out[k].v = (int64_t)(R - 1) * C + j; out[k].kind = 0; out[k].e = (int64_t)(m - 1) * (n - 1) + j; out[k].delta = -1; k++;
    }
    for (int i = 0; i < R; i++) {  /* left edges vy(i,0): ground -> p(i,0) rightward: -1 */
        out[k].v = (int64_t)i * C; out[k].kind = 1; out[k].e = (int64_t)i * n; out[k].delta = -1; k++;
    }
    for (int i = 0; i < R; i++) {  /* right edges vy(i,n-1): ground -> p(i,C-1) leftward: +1 */
        out[k].v = (int64_t)i * C + C - 1; out[k].kind = 1; out[k].e = (int64_t)i * n + n - 1; out[k].delta = +1; k++;
    }
    return k;
}

static int arc_cost(const graph *g, const arc *a, int64_t *cost) {
    int f = a->kind == 0 ? g->fx[a->e] : g->fy[a->e];
    int cp = a->kind == 0 ? g->cxp[a->e] : g->cyp[a->e];
    int cn = a->kind == 0 ? g->cxn[a->e] : g->cyn[a->e];
    return move_cost(f, a->delta, cp, cn, cost);
}

static void apply_move(graph *g, const arc *a) {
    if (a->kind == 0) g->fx[a->e] += a->delta;
    else g->fy[a->e] += a->delta;
}

/* binary min-heap of (dist, node) with lazy deletion */
typedef struct { int64_t d, v; } hent;
typedef struct { hent *a; int64_t n, cap; } heap;

static int hless(hent x, hent y) { return x.d < y.d || (x.d == y.d && x.v < y.v); }
static int hpush(heap *h, int64_t d, int64_t v) {
    if (h->n == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 1024;
        hent *na = realloc(h->a, sizeof(hent) * nc);
        if (!na) return -1;
        h->a = na; h->cap = nc;
    }
    int64_t i = h->n++;
    h->a[i].d = d; h->a[i].v = v;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!hless(h->a[i], h->a[p])) break;
        hent t = h->a[i]; h->a[i] = h->a[p]; h->a[p] = t; i = p;
    }
    return 0;
}
static hent hpop(heap *h) {
    hent top = h->a[0];
    h->a[0] = h->a[--h->n];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, s = i;
        if (l < h->n && hless(h->a[l], h->a[s])) s = l;
        if (r < h->n && hless(h->a[r], h->a[s])) s = r;
        if (s == i) break;
        hent t = h->a[i]; h->a[i] = h->a[s]; h->a[s] = t; i = s;
    }
    return top;
}

/* Successive shortest paths.  res: loop residues; outputs dk_x [m*(n-1)],
 * dk_y [(m-1)*n] in {-1,0,1}, pot [(m-1)(n-1)+1] int64 (nullable) and the
 * total cost.  stats (nullable): [0]=augmentations, [1]=settled nodes summed
 * over searches, [2]=arcs scanned.  Pinned by brute-force enumeration, an LP
 * solver, network simplex and the self-certificate. */
int wwo_mcf(const int8_t *res, int m, int n, const int16_t *cxp, const int16_t *cxn,
            const int16_t *cyp, const int16_t *cyn, int8_t *dk_x, int8_t *dk_y,
            int64_t *pot_out, int64_t *total, int64_t *stats) {
    if (m < 1 || n < 1) return WWO_E_INVALID_ARG;
    int64_t nxe = (int64_t)m * (n - 1), nye = (int64_t)(m - 1) * n;
    if (n < 2) nxe = 0;
    if (m < 2) nye = 0;
    for (int64_t e = 0; e < nxe; e++) dk_x[e] = 0;
    for (int64_t e = 0; e < nye; e++) dk_y[e] = 0;
    if (m < 2 || n < 2) {
        if (pot_out) pot_out[0] = 0;
        *total = 0;
        if (stats) { stats[0] = stats[1] = stats[2] = 0; }
        return WWO_OK;
    }
    graph g;
    g.m = m; g.n = n; g.R = m - 1; g.C = n - 1;
    g.G = (int64_t)g.R * g.C; g.nn = g.G + 1;
    g.cxp = cxp; g.cxn = cxn; g.cyp = cyp; g.cyn = cyn;
    g.fx = dk_x; g.fy = dk_y;
    int64_t nn = g.nn;
    int64_t *ex = calloc(nn, sizeof(int64_t));
    int64_t *pot = calloc(nn, sizeof(int64_t));
    int64_t *dist = malloc(sizeof(int64_t) * nn);
    int64_t *pred = malloc(sizeof(int64_t) * nn);     /* predecessor node */
    arc *parc = malloc(sizeof(arc) * nn);              /* arc used to reach node */
    uint8_t *state = calloc(nn, 1);                    /* 0 untouched, 1 labelled, 2 settled */
    int64_t *touched = malloc(sizeof(int64_t) * nn);
    int64_t gdeg = 2 * (int64_t)g.C + 2 * (int64_t)g.R;
    arc *arcs = malloc(sizeof(arc) * (gdeg > 4 ? gdeg : 4));
    heap hp = {0, 0, 0};
    if (!ex || !pot || !dist || !pred || !parc || !state || !touched || !arcs) {
        free(ex); free(pot); free(dist); free(pred); free(parc); free(state); free(touched); free(arcs);
        return WWO_E_OOM;
    }
    int64_t tot = 0;
    for (int64_t u = 0; u < g.G; u++) { ex[u] = res[u]; tot += res[u]; }
    ex[g.G] = -tot;
    int64_t n_aug = 0, n_settled = 0, n_scan = 0;
    int rc = WWO_OK;
    int64_t src = 0;
    for (;;) {
        while (src < nn && ex[src] <= 0) src++;
        if (src >= nn) break;
        /* Dijkstra from src over reduced costs until the first deficit */
        int64_t ntouch = 0;
        hp.n = 0;
        dist[src] = 0; pred[src] = -1; state[src] = 1; touched[ntouch++] = src;
        if (hpush(&hp, 0, src)) { rc = WWO_E_OOM; break; }
        int64_t t = -1;
        while (hp.n > 0) {
            hent top = hpop(&hp);
            int64_t u = top.v;
            if (state[u] == 2 || top.d != dist[u]) continue;
            state[u] = 2;
            n_settled++;
            if (ex[u] < 0) { t = u; break; }
            int na = out_arcs(&g, u, arcs);
            for (int a = 0; a < na; a++) {
                int64_t c;
                if (arc_cost(&g, &arcs[a], &c)) continue;
                n_scan++;
                int64_t v = arcs[a].v;
                if (state[v] == 2) continue;
                int64_t rcst = c - pot[u] + pot[v];
                int64_t nd = dist[u] + rcst;
                if (state[v] == 0 || nd < dist[v]) {
                    if (state[v] == 0) { state[v] = 1; touched[ntouch++] = v; }
                    dist[v] = nd; pred[v] = u; parc[v] = arcs[a];
                    if (hpush(&hp, nd, v)) { rc = WWO_E_OOM; break; }
                }
            }
            if (rc) break;
        }
        if (rc) break;
        if (t < 0) { rc = WWO_E_INFEASIBLE; break; }
        /* potentials of settled nodes: pi(v) += d(t) - d(v) */
        int64_t dt = dist[t];
        for (int64_t k = 0; k < ntouch; k++) {
            int64_t v = touched[k];
            if (state[v] == 2) pot[v] += dt - dist[v];
        }
        /* augment one unit along the predecessor path */
        for (int64_t v = t; v != src; v = pred[v]) apply_move(&g, &parc[v]);
        ex[src]--; ex[t]++;
        n_aug++;
        for (int64_t k = 0; k < ntouch; k++) state[touched[k]] = 0;
    }
    if (rc == WWO_OK) {
        int64_t cost = 0;
        for (int64_t e = 0; e < nxe; e++) cost += dk_x[e] > 0 ? cxp[e] : (dk_x[e] < 0 ? cxn[e] : 0);
        for (int64_t e = 0; e < nye; e++) cost += dk_y[e] > 0 ? cyp[e] : (dk_y[e] < 0 ? cyn[e] : 0);
        *total = cost;
        if (pot_out) memcpy(pot_out, pot, sizeof(int64_t) * nn);
        if (stats) { stats[0] = n_aug; stats[1] = n_settled; stats[2] = n_scan; }
    }
    free(hp.a);
    free(ex); free(pot); free(dist); free(pred); free(parc); free(state); free(touched); free(arcs);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Optimality certificate and O6 uniqueness certificate                      */
/* ------------------------------------------------------------------------ */

/* Check that (dk, pot) is an optimal flow: divergence equals the residues at
 * every loop node (and the balancing charge at the ground), every residual arc
 * has reduced cost c - pot(u) + pot(v) >= 0, and |dk| <= 1.  out (nullable):
 * [0] = number of divergence violations, [1] = number of negative reduced
 * costs, [2] = minimum reduced cost seen.  Returns WWO_OK or WWO_E_CERT. */
int wwo_check_optimal(const int8_t *res, int m, int n, const int16_t *cxp, const int16_t *cxn,
                      const int16_t *cyp, const int16_t *cyn, const int8_t *dk_x,
                      const int8_t *dk_y, const int64_t *pot, int64_t *out) {
    if (m < 2 || n < 2) return WWO_OK;
    graph g;
    g.m = m; g.n = n; g.R = m - 1; g.C = n - 1;
    g.G = (int64_t)g.R * g.C; g.nn = g.G + 1;
    g.cxp = cxp; g.cxn = cxn; g.cyp = cyp; g.cyn = cyn;
    g.fx = (int8_t *)dk_x; g.fy = (int8_t *)dk_y;
    int64_t *div = calloc(g.nn, sizeof(int64_t));
    int64_t gdeg = 2 * (int64_t)g.C + 2 * (int64_t)g.R;
    arc *arcs = malloc(sizeof(arc) * (gdeg > 4 ? gdeg : 4));
    if (!div || !arcs) { free(div); free(arcs); return WWO_E_OOM; }
    int64_t nbad_div = 0, nneg = 0, minrc = INT64_MAX;
    int64_t nxe = (int64_t)m * (n - 1), nye = (int64_t)(m - 1) * n;
    for (int64_t e = 0; e < nxe; e++) if (dk_x[e] < -1 || dk_x[e] > 1) nbad_div++;
    for (int64_t e = 0; e < nye; e++) if (dk_y[e] < -1 || dk_y[e] > 1) nbad_div++;
    for (int64_t u = 0; u < g.nn; u++) {
        int na = out_arcs(&g, u, arcs);
        for (int a = 0; a < na; a++) {
            int64_t c;
            if (!arc_cost(&g, &arcs[a], &c)) {
                int64_t rc = c - pot[u] + pot[arcs[a].v];
                if (rc < minrc) minrc = rc;
                if (rc < 0) nneg++;
            }
        }
    }
    /* divergence: out-flow of loop u across each of its edges.  A +1 cycle
     * difference on an edge carries one unit along the arc whose move is +1. */
    for (int64_t u = 0; u < g.G; u++) {
        int na = out_arcs(&g, u, arcs);
        int64_t s = 0;
        for (int a = 0; a < na; a++) {
            int f = arcs[a].kind == 0 ? dk_x[arcs[a].e] : dk_y[arcs[a].e];
            s += (int64_t)f * arcs[a].delta;
        }
        div[u] = s;
    }
    int64_t tot = 0;
    for (int64_t u = 0; u < g.G; u++) { if (div[u] != res[u]) nbad_div++; tot += res[u]; }
    {
        int na = out_arcs(&g, g.G, arcs);
        int64_t s = 0;
        for (int a = 0; a < na; a++) {
            int f = arcs[a].kind == 0 ? dk_x[arcs[a].e] : dk_y[arcs[a].e];
            s += (int64_t)f * arcs[a].delta;
        }
        if (s != -tot) nbad_div++;
    }
    if (out) { out[0] = nbad_div; out[1] = nneg; out[2] = minrc; }
    free(div); free(arcs);
    return (nbad_div == 0 && nneg == 0) ? WWO_OK : WWO_E_CERT;
}

/* Edges whose cycle difference is the same in every optimal flow: build the
 * subgraph of residual arcs with zero reduced cost under pot, find its
 * strongly connected components (iterative Tarjan); an edge is fixed iff none
 * of its zero-reduced-cost residual arcs lies on a cycle of that subgraph
 * that uses the edge once (two optima differ by such cycles, by
 * complementary slackness).
 * fixed_x [m*(n-1)], fixed_y [(m-1)*n] get 1 for fixed edges. */
int wwo_fixed_edges(int m, int n, const int16_t *cxp, const int16_t *cxn, const int16_t *cyp,
                    const int16_t *cyn, const int8_t *dk_x, const int8_t *dk_y, const int64_t *pot,
                    uint8_t *fixed_x, uint8_t *fixed_y) {
    int64_t nxe = (int64_t)m * (n - 1), nye = (int64_t)(m - 1) * n;
    if (n < 2) nxe = 0;
    if (m < 2) nye = 0;
    for (int64_t e = 0; e < nxe; e++) fixed_x[e] = 1;
    for (int64_t e = 0; e < nye; e++) fixed_y[e] = 1;
    if (m < 2 || n < 2) {
        /* no loops: every edge is a ground-to-ground self-loop, a cycle on
         * its own, so it changes iff one of its moves costs nothing */
        for (int64_t e = 0; e < nxe; e++) {
            int64_t c;
            int f = dk_x[e];
            if ((!move_cost(f, 1, cxp[e], cxn[e], &c) && c == 0) ||
                (!move_cost(f, -1, cxp[e], cxn[e], &c) && c == 0)) fixed_x[e] = 0;
        }
        for (int64_t e = 0; e < nye; e++) {
            int64_t c;
            int f = dk_y[e];
            if ((!move_cost(f, 1, cyp[e], cyn[e], &c) && c == 0) ||
                (!move_cost(f, -1, cyp[e], cyn[e], &c) && c == 0)) fixed_y[e] = 0;
        }
        return WWO_OK;
    }
    graph g;
    g.m = m; g.n = n; g.R = m - 1; g.C = n - 1;
    g.G = (int64_t)g.R * g.C; g.nn = g.G + 1;
    g.cxp = cxp; g.cxn = cxn; g.cyp = cyp; g.cyn = cyn;
    g.fx = (int8_t *)dk_x; g.fy = (int8_t *)dk_y;
    int64_t nn = g.nn;
    int64_t gdeg = 2 * (int64_t)g.C + 2 * (int64_t)g.R;
    /* zero-reduced-cost residual adjacency in CSR form */
    int64_t *off = calloc(nn + 1, sizeof(int64_t));
    arc *arcs = malloc(sizeof(arc) * (gdeg > 4 ? gdeg : 4));
    if (!off || !arcs) { free(off); free(arcs); return WWO_E_OOM; }
    for (int64_t u = 0; u < nn; u++) {
        int na = out_arcs(&g, u, arcs);
        for (int a = 0; a < na; a++) {
            int64_t c;
            if (!arc_cost(&g, &arcs[a], &c) && c - pot[u] + pot[arcs[a].v] == 0) off[u + 1]++;
        }
    }
    for (int64_t u = 0; u < nn; u++) off[u + 1] += off[u];
    int64_t *adj = malloc(sizeof(int64_t) * (off[nn] ? off[nn] : 1));
    int64_t *fill = malloc(sizeof(int64_t) * nn);
    if (!adj || !fill) { free(off); free(arcs); free(adj); free(fill); return WWO_E_OOM; }
    memcpy(fill, off, sizeof(int64_t) * nn);
    for (int64_t u = 0; u < nn; u++) {
        int na = out_arcs(&g, u, arcs);
        for (int a = 0; a < na; a++) {
            int64_t c;
            if (!arc_cost(&g, &arcs[a], &c) && c - pot[u] + pot[arcs[a].v] == 0) adj[fill[u]++] = arcs[a].v;
        }
    }
    /* iterative Tarjan */
    int64_t *idx = malloc(sizeof(int64_t) * nn), *low = malloc(sizeof(int64_t) * nn);
    int64_t *comp = malloc(sizeof(int64_t) * nn), *stk = malloc(sizeof(int64_t) * nn);
    int64_t *cs_node = malloc(sizeof(int64_t) * nn), *cs_it = malloc(sizeof(int64_t) * nn);
    uint8_t *onstk = calloc(nn, 1);
    if (!idx || !low || !comp || !stk || !cs_node || !cs_it || !onstk) {
        free(off); free(arcs); free(adj); free(fill); free(idx); free(low); free(comp);
        free(stk); free(cs_node); free(cs_it); free(onstk);
        return WWO_E_OOM;
    }
    for (int64_t u = 0; u < nn; u++) idx[u] = -1;
    int64_t counter = 0, sp = 0, ncomp = 0;
    for (int64_t s = 0; s < nn; s++) {
        if (idx[s] >= 0) continue;
        int64_t csp = 0;
        cs_node[csp] = s; cs_it[csp] = off[s]; csp++;
        idx[s] = low[s] = counter++; stk[sp++] = s; onstk[s] = 1;
        while (csp > 0) {
            int64_t u = cs_node[csp - 1];
            if (cs_it[csp - 1] < off[u + 1]) {
                int64_t v = adj[cs_it[csp - 1]++];
                if (idx[v] < 0) {
                    idx[v] = low[v] = counter++; stk[sp++] = v; onstk[v] = 1;
                    cs_node[csp] = v; cs_it[csp] = off[v]; csp++;
                } else if (onstk[v] && idx[v] < low[u]) low[u] = idx[v];
            } else {
                if (low[u] == idx[u]) {
                    int64_t w;
                    do { w = stk[--sp]; onstk[w] = 0; comp[w] = ncomp; } while (w != u);
                    ncomp++;
                }
                csp--;
                if (csp > 0) {
                    int64_t p = cs_node[csp - 1];
                    if (low[u] < low[p]) low[p] = low[u];
                }
            }
        }
    }
    /* An edge changes between optima iff one of its zero-reduced-cost
     * residual arcs u->v closes a cycle v ~> u that does not use the same
     * edge again (a cycle through both moves of one edge changes nothing).
     * Within one component that is automatic unless both moves of the edge
     * have zero reduced cost; then search v ~> u without that edge. */
    int64_t *stamp = malloc(sizeof(int64_t) * nn), *bq = malloc(sizeof(int64_t) * nn);
    arc *arcs2 = malloc(sizeof(arc) * (gdeg > 4 ? gdeg : 4));
    if (!stamp || !bq || !arcs2) {
        free(stamp); free(bq); free(arcs2);
        free(off); free(arcs); free(adj); free(fill); free(idx); free(low); free(comp);
        free(stk); free(cs_node); free(cs_it); free(onstk);
        return WWO_E_OOM;
    }
    for (int64_t u = 0; u < nn; u++) stamp[u] = -1;
    int64_t query = 0;
    for (int64_t u = 0; u < nn; u++) {
        int na = out_arcs(&g, u, arcs);
        for (int a = 0; a < na; a++) {
            int64_t c, v = arcs[a].v;
            if (arc_cost(&g, &arcs[a], &c)) continue;
            if (c - pot[u] + pot[v] != 0) continue;
            if (comp[u] != comp[v]) continue;
            int kind = arcs[a].kind;
            int64_t e = arcs[a].e;
            if ((kind == 0 ? fixed_x[e] : fixed_y[e]) == 0) continue;
            /* does the opposite move of this edge also have zero reduced cost? */
            arc rev = arcs[a];
            rev.v = u; rev.delta = -arcs[a].delta;
            int64_t cr;
            int dbl = !arc_cost(&g, &rev, &cr) && cr - pot[v] + pot[u] == 0;
            int changes = 1;
            if (dbl) {
                /* breadth-first search v ~> u over zero-reduced-cost residual
                 * arcs, never using edge (kind, e) */
                changes = 0;
                int64_t h = 0, t = 0;
                bq[t++] = v; stamp[v] = query;
                while (h < t && !changes) {
                    int64_t x = bq[h++];
                    int nb = out_arcs(&g, x, arcs2);
                    for (int b = 0; b < nb; b++) {
                        if (arcs2[b].kind == kind && arcs2[b].e == e) continue;
                        int64_t cb, y = arcs2[b].v;
                        if (arc_cost(&g, &arcs2[b], &cb)) continue;
                        if (cb - pot[x] + pot[y] != 0) continue;
                        if (y == u) { changes = 1; break; }
                        if (stamp[y] == query) continue;
                        stamp[y] = query;
                        bq[t++] = y;
                    }
                }
                query++;
            }
            if (changes) {
                if (kind == 0) fixed_x[e] = 0;
                else fixed_y[e] = 0;
            }
        }
    }
    free(stamp); free(bq); free(arcs2);
    free(off); free(arcs); free(adj); free(fill); free(idx); free(low); free(comp);
    free(stk); free(cs_node); free(cs_it); free(onstk);
    return WWO_OK;
}

/* ------------------------------------------------------------------------ */
/* O7  integration of the corrected gradients (Section II-A, II-C)          */
/* ------------------------------------------------------------------------ */

/* K(ref) = 0; K grows by dk_e - w_e along every edge, first down column 0,
 * then along each row; phi = psi + 2 pi K in double, rounded to float32, and
 * nodata where invalid.  ref_i < 0 selects the first valid pixel row-major.
 * Pinned by path independence, congruence and exact recovery of smooth
 * residue-free fields. */
int wwo_integrate(const float *psi, const uint8_t *valid, const int8_t *dk_x, const int8_t *dk_y,
                  int m, int n, int ref_i, int ref_j, float nodata, int32_t *K, float *phi) {
    if (m < 1 || n < 1) return WWO_E_INVALID_ARG;
    int64_t N = (int64_t)m * n, ref = 0;
    if (ref_i < 0) {
        ref = 0;
        if (valid) {
            int64_t k = 0;
            while (k < N && !valid[k]) k++;
            ref = k < N ? k : 0;
        }
    } else {
        if (ref_i >= m || ref_j < 0 || ref_j >= n) return WWO_E_INVALID_ARG;
        ref = (int64_t)ref_i * n + ref_j;
    }
    K[0] = 0;
    for (int i = 1; i < m; i++)
        K[(int64_t)i * n] = K[(int64_t)(i - 1) * n] + dk_y[(int64_t)(i - 1) * n] - wy(psi, valid, n, i - 1, 0);
    for (int i = 0; i < m; i++)
        for (int j = 1; j < n; j++) {
            int64_t a = (int64_t)i * n + j;
            K[a] = K[a - 1] + dk_x[(int64_t)i * (n - 1) + j - 1] - wx(psi, valid, n, i, j - 1);
        }
    int32_t k0 = K[ref];
    for (int64_t a = 0; a < N; a++) {
        K[a] -= k0;
        if (valid && !valid[a]) phi[a] = nodata;
        else phi[a] = (float)((double)psi[a] + TWO_PI_D * (double)K[a]);
    }
    return WWO_OK;
}

/* Pixels whose K is the same in every optimum given K(ref) = 0: those joined
 * to ref by fixed edges.  comp (nullable) receives a label per pixel of its
 * fixed-edge component (the component of ref is 0). */
int wwo_certified_pixels(int m, int n, const uint8_t *fixed_x, const uint8_t *fixed_y, int64_t ref,
                         uint8_t *cert, int64_t *comp) {
    int64_t N = (int64_t)m * n;
    int64_t *lab = malloc(sizeof(int64_t) * N), *q = malloc(sizeof(int64_t) * N);
    if (!lab || !q) { free(lab); free(q); return WWO_E_OOM; }
    for (int64_t a = 0; a < N; a++) lab[a] = -1;
    int64_t next = 0;
    for (int64_t pass = -1; pass < N; pass++) {
        int64_t s = pass < 0 ? ref : pass;
        if (lab[s] >= 0) continue;
        int64_t h = 0, t = 0;
        q[t++] = s; lab[s] = next;
        while (h < t) {
            int64_t a = q[h++];
            int i = (int)(a / n), j = (int)(a % n);
            if (j + 1 < n && fixed_x[(int64_t)i * (n - 1) + j] && lab[a + 1] < 0) { lab[a + 1] = next; q[t++] = a + 1; }
            if (j > 0 && fixed_x[(int64_t)i * (n - 1) + j - 1] && lab[a - 1] < 0) { lab[a - 1] = next; q[t++] = a - 1; }
            if (i + 1 < m && fixed_y[(int64_t)i * n + j] && lab[a + n] < 0) { lab[a + n] = next; q[t++] = a + n; }
            if (i > 0 && fixed_y[(int64_t)(i - 1) * n + j] && lab[a - n] < 0) { lab[a - n] = next; q[t++] = a - n; }
        }
        next++;
    }
    for (int64_t a = 0; a < N; a++) {
        cert[a] = lab[a] == 0;
        if (comp) comp[a] = lab[a];
    }
    free(lab); free(q);
    return WWO_OK;
}

/* ------------------------------------------------------------------------ */
/* O8  brute force over K (tests only, at most 16 pixels)                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    int m, n;
    const int8_t *wxa, *wya;      /* wrap counts per edge */
    const int16_t *cxp, *cxn, *cyp, *cyn;
    int32_t K[16];
    int64_t best, count;
} bf_state;

static int64_t bf_edge(int dk, int cp, int cn) { return dk > 0 ? cp : (dk < 0 ? cn : 0); }

static void bf_rec(bf_state *s, int a, int64_t cost) {
    int N = s->m * s->n;
    if (cost > s->best) return;
    if (a == N) {
        if (cost < s->best) { s->best = cost; s->count = 1; }
        else s->count++;
        return;
    }
    int i = a / s->n, j = a % s->n;
    int lo = -1000000, hi = 1000000;
    /* |K_v - K_u + w| <= 1 for the left and up neighbours */
    if (j > 0) {
        int w = s->wxa[i * (s->n - 1) + j - 1];
        int base = s->K[a - 1] - w;
        if (base - 1 > lo) lo = base - 1;
        if (base + 1 < hi) hi = base + 1;
    }
    if (i > 0) {
        int w = s->wya[(i - 1) * s->n + j];
        int base = s->K[a - s->n] - w;
        if (base - 1 > lo) lo = base - 1;
        if (base + 1 < hi) hi = base + 1;
    }
    for (int k = lo; k <= hi; k++) {
        int64_t c = cost;
        if (j > 0) {
            int e = i * (s->n - 1) + j - 1;
            c += bf_edge(k - s->K[a - 1] + s->wxa[e], s->cxp[e], s->cxn[e]);
        }
        if (i > 0) {
            int e = (i - 1) * s->n + j;
            c += bf_edge(k - s->K[a - s->n] + s->wya[e], s->cyp[e], s->cyn[e]);
        }
        s->K[a] = k;
        bf_rec(s, a + 1, c);
    }
}

/* Minimum of sum_e C_e(K_v - K_u + w_e) over integer K with K(0,0) = 0 and
 * every |K_v - K_u + w_e| <= 1, and the number of minimising K fields.  The
 * wrap counts wx [m*(n-1)], wy [(m-1)*n] are inputs (so that tests can pick
 * arbitrary residue patterns). */
int wwo_bruteforce(int m, int n, const int8_t *wxa, const int8_t *wya, const int16_t *cxp,
                   const int16_t *cxn, const int16_t *cyp, const int16_t *cyn,
                   int64_t *best, int64_t *count) {
    if (m < 1 || n < 1 || m * n > 16) return WWO_E_INVALID_ARG;
    bf_state s;
    s.m = m; s.n = n; s.wxa = wxa; s.wya = wya;
    s.cxp = cxp; s.cxn = cxn; s.cyp = cyp; s.cyn = cyn;
    s.best = INT64_MAX; s.count = 0;
    s.K[0] = 0;
    bf_rec(&s, 1, 0);
    *best = s.best;
    *count = s.count;
    return s.count > 0 ? WWO_OK : WWO_E_INFEASIBLE;
}

/* ------------------------------------------------------------------------ */
/* Connected components of reliably unwrapped pixels (Section II-D)         */
/* ------------------------------------------------------------------------ */

/* An edge is reliable when both of its pixels are valid and changing its
 * cycle difference dk by +1 or by -1 would each raise that edge's cost by
 * more than `threshold`: with dk = 0 this means c+ > threshold and
 * c- > threshold; with dk = +-1 one of the two changes would refund the
 * edge's cost (never a rise), so such an edge is not reliable. */
static int cc_reliable(int8_t dk, int16_t cp, int16_t cn, int threshold) {
    return dk == 0 && cp > threshold && cn > threshold;
}

/* Grows components over reliable edges by breadth-first search from every
 * not yet labelled valid pixel in row-major order, so components are
 * discovered in the order of their first pixel.  Components with fewer than
 * min_size pixels, and invalid pixels, get label 0; the others are numbered
 * 1, 2, ... in discovery order.  labels uint32 [m*n]; *ncomp = number of
 * labelled components.  valid NULL = all valid. */
int wwo_connected_components(const int8_t *dk_x, const int8_t *dk_y, const int16_t *cxp,
                             const int16_t *cxn, const int16_t *cyp, const int16_t *cyn,
                             const uint8_t *valid, int m, int n, int threshold, int64_t min_size,
                             uint32_t *labels, int64_t *ncomp) {
    if (m < 1 || n < 1 || min_size < 1) return WWO_E_INVALID_ARG;
    const int64_t N = (int64_t)m * n;
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    int64_t *comp = (int64_t *)malloc(sizeof(int64_t) * (size_t)N); /* discovery index */
    int64_t *size = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    if (!queue || !comp || !size) {
        free(queue); free(comp); free(size);
        return WWO_E_OOM;
    }
    for (int64_t p = 0; p < N; p++) comp[p] = -1;
    int64_t ncomp_all = 0;
    for (int64_t s = 0; s < N; s++) {
        if (comp[s] >= 0 || (valid && !valid[s])) continue;
        const int64_t c = ncomp_all++;
        int64_t head = 0, tail = 0;
        queue[tail++] = s;
        comp[s] = c;
        while (head < tail) {
            const int64_t p = queue[head++];
            const int i = (int)(p / n), j = (int)(p % n);
            /* the four edges of pixel p and the pixel across each */
            for (int d = 0; d < 4; d++) {
                int64_t q, e;
                int rel;
                if (d == 0) {        /* right: hx(i, j) */
                    if (j + 1 >= n) continue;
                    q = p + 1;
                    e = (int64_t)i * (n - 1) + j;
                    rel = cc_reliable(dk_x[e], cxp[e], cxn[e], threshold);
                } else if (d == 1) { /* left: hx(i, j-1) */
                    if (j == 0) continue;
                    q = p - 1;
                    e = (int64_t)i * (n - 1) + j - 1;
                    rel = cc_reliable(dk_x[e], cxp[e], cxn[e], threshold);
                } else if (d == 2) { /* down: vy(i, j) */
                    if (i + 1 >= m) continue;
                    q = p + n;
                    e = (int64_t)i * n + j;
                    rel = cc_reliable(dk_y[e], cyp[e], cyn[e], threshold);
                } else {             /* up: vy(i-1, j) */
                    if (i == 0) continue;
                    q = p - n;
                    e = (int64_t)(i - 1) * n + j;
                    rel = cc_reliable(dk_y[e], cyp[e], cyn[e], threshold);
                }
                if (!rel || comp[q] >= 0 || (valid && !valid[q])) continue;
                comp[q] = c;
                queue[tail++] = q;
            }
        }
        size[c] = tail;
    }
    /* number the components that are large enough, in discovery order */
    int64_t next = 0;
    for (int64_t c = 0; c < ncomp_all; c++) size[c] = size[c] >= min_size ? ++next : 0;
    for (int64_t p = 0; p < N; p++) labels[p] = comp[p] >= 0 ? (uint32_t)size[comp[p]] : 0u;
    *ncomp = next;
    free(queue); free(comp); free(size);
    return WWO_OK;
}
