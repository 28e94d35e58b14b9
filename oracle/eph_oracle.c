/*
 * Plain FP64 CPU oracle for the e-ph collision integral.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * library never does, and the two share no code.
 *
 * What it computes (paper: Results, "Collision integral, e-ph coupling matrix,
 * and scattering channels", Eq. 2).  For a state d = |n k> and a partner
 * p = |m k+q> joined by phonon mode nu at wave vector q,
 *
 *   T(d,p) = -(2 pi / hbar)(1/N_q) |g|^2 [ G(e_d - e_p + hw) F_abs
 *                                         + G(e_d - e_p - hw) F_em ]
 *   F_abs  = f_d (1 - f_p) N - f_p (1 - f_d) (N + 1)
 *   F_em   = f_d (1 - f_p) (N + 1) - f_p (1 - f_d) N
 *
 * with G a normalised Gaussian of standard deviation sigma, N = N_{nu q} the
 * phonon occupation and hw = hbar omega_{nu q}.  The paper defers F_abs and
 * F_em to a Methods section that is not part of the text; the forms above are
 * Fermi's golden rule for absorption (d absorbs a phonon, N) and emission
 * (d emits, N + 1), each minus its reverse process.
 *
 * Each scattering channel (an unordered state pair {i, j} plus a mode) enters
 * I(i) with partner j and I(j) with partner i (Optimized GPU algorithm, step 1:
 * one channel feeds two collision-integral elements).  The channel-list loop
 * below evaluates BOTH orientations from the formula, each with its own q
 * (k_j - k_i for i's view, k_i - k_j for j's view); it does not assume that
 * the two are opposite.  Tests check that they are.
 *
 * Momentum conservation: q is the q-grid vector (k_p - k_d) / r with
 * r = Nk / Nq per direction (commensurate grids).
 *
 * Constants: hbar = 0.6582119569 eV fs (CODATA 2018).  Units: eV, fs.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_HBAR_EV_FS 0.6582119569
#define ORC_PI 3.14159265358979323846

typedef struct {
    int n_states;
    const int32_t *state_k;
    const double *eps;
    int kgrid[3];
    int qgrid[3];
    int n_modes;
    const double *hw;   /* [Nq][n_modes] */
    const double *nph;  /* [Nq][n_modes] */
    double sigma;
    double n_q_norm;
} orc_sys;

static void k_coords(int lin, const int g[3], int c[3]) {
    c[2] = lin % g[2];
    lin /= g[2];
    c[1] = lin % g[1];
    c[0] = lin / g[1];
}

/* linear q index of k_p - k_d on the q grid */
static int q_index(const orc_sys *s, int d, int p) {
    int cd[3], cp[3], q[3];
    k_coords(s->state_k[d], s->kgrid, cd);
    k_coords(s->state_k[p], s->kgrid, cp);
    for (int a = 0; a < 3; ++a) {
        int r = s->kgrid[a] / s->qgrid[a];
        int dk = ((cp[a] - cd[a]) % s->kgrid[a] + s->kgrid[a]) % s->kgrid[a];
        q[a] = dk / r;
    }
    return (q[0] * s->qgrid[1] + q[1]) * s->qgrid[2] + q[2];
}

static double gauss(double x, double sigma) {
    return exp(-x * x / (2.0 * sigma * sigma)) / (sigma * sqrt(2.0 * ORC_PI));
}

/* Eq. 2 summand for destination d and partner p through mode nu, with |g|^2 = g2 */
static double eq2_term(const orc_sys *s, const double *f, int d, int p, int nu, double g2) {
    int q = q_index(s, d, p);
    double w = s->hw[(long)q * s->n_modes + nu];
    double N = s->nph[(long)q * s->n_modes + nu];
    double fd = f[d], fp = f[p];
    double F_abs = fd * (1.0 - fp) * N - fp * (1.0 - fd) * (N + 1.0);
    double F_em = fd * (1.0 - fp) * (N + 1.0) - fp * (1.0 - fd) * N;
    double de = s->eps[d] - s->eps[p];
    double pref = 2.0 * ORC_PI / ORC_HBAR_EV_FS / s->n_q_norm;
    return -pref * g2 * (gauss(de + w, s->sigma) * F_abs + gauss(de - w, s->sigma) * F_em);
}

static orc_sys make_sys(int n_states, const int32_t *state_k, const double *eps,
                        const int32_t *kgrid, const int32_t *qgrid, int n_modes,
                        const double *hw, const double *nph, double sigma, double n_q_norm) {
    orc_sys s;
    s.n_states = n_states;
    s.state_k = state_k;
    s.eps = eps;
    for (int a = 0; a < 3; ++a) {
        s.kgrid[a] = kgrid[a];
        s.qgrid[a] = qgrid[a];
    }
    s.n_modes = n_modes;
    s.hw = hw;
    s.nph = nph;
    s.sigma = sigma;
    s.n_q_norm = n_q_norm;
    return s;
}

/*
 * Collision integral I[f] over a channel list, looped once in list order,
 * sequentially (the Baseline-CPU loop shape of the paper's reference CPU
 * algorithm, without threads and therefore without atomics).
 * If mask is non-NULL, only destinations with mask[d] != 0 are accumulated
 * (the others are left at 0); this evaluates sampled outputs of a large case.
 */
void orc_collision(int n_states, const int32_t *state_k, const double *eps,
                   const int32_t *kgrid, const int32_t *qgrid, int n_modes,
                   const double *hw, const double *nph, double sigma, double n_q_norm,
                   int64_t n_ch, const int32_t *ch_i, const int32_t *ch_j,
                   const int8_t *ch_nu, const double *g2, const double *f,
                   const uint8_t *mask, double *I) {
    orc_sys s = make_sys(n_states, state_k, eps, kgrid, qgrid, n_modes, hw, nph, sigma, n_q_norm);
    memset(I, 0, sizeof(double) * (size_t)n_states);
    for (int64_t c = 0; c < n_ch; ++c) {
        int i = ch_i[c], j = ch_j[c], nu = ch_nu[c];
        if (!mask || mask[i]) I[i] += eq2_term(&s, f, i, j, nu, g2[c]);
        if (!mask || mask[j]) I[j] += eq2_term(&s, f, j, i, nu, g2[c]);
    }
}

/*
 * Reverse mode of L = sum_d lam_d I_d, derived by hand from eq2_term:
 *   dT(d,p)/df_d = -P g2 [Ga ((1-f_p) N + f_p (N+1)) + Ge ((1-f_p)(N+1) + f_p N)]
 *   dT(d,p)/df_p = +P g2 [Ga (f_d N + (1-f_d)(N+1)) + Ge (f_d (N+1) + (1-f_d) N)]
 *   dT(d,p)/dg2  = T(d,p) / g2
 * with P = 2 pi / (hbar N_q), Ga = G(e_d - e_p + hw), Ge = G(e_d - e_p - hw).
 * gf [S] and gg2 [n_ch] are overwritten; either may be NULL.
 */
static void term_grads(const orc_sys *s, const double *f, int d, int p, int nu, double g2,
                       double *dfd, double *dfp, double *dg2) {
    int q = q_index(s, d, p);
    double w = s->hw[(long)q * s->n_modes + nu];
    double N = s->nph[(long)q * s->n_modes + nu];
    double fd = f[d], fp = f[p];
    double de = s->eps[d] - s->eps[p];
    double P = 2.0 * ORC_PI / ORC_HBAR_EV_FS / s->n_q_norm;
    double Ga = gauss(de + w, s->sigma), Ge = gauss(de - w, s->sigma);
    double F_abs = fd * (1.0 - fp) * N - fp * (1.0 - fd) * (N + 1.0);
    double F_em = fd * (1.0 - fp) * (N + 1.0) - fp * (1.0 - fd) * N;
    *dfd = -P * g2 * (Ga * ((1.0 - fp) * N + fp * (N + 1.0)) + Ge * ((1.0 - fp) * (N + 1.0) + fp * N));
    *dfp = P * g2 * (Ga * (fd * N + (1.0 - fd) * (N + 1.0)) + Ge * (fd * (N + 1.0) + (1.0 - fd) * N));
    *dg2 = -P * (Ga * F_abs + Ge * F_em);
}

void orc_collision_vjp(int n_states, const int32_t *state_k, const double *eps,
                       const int32_t *kgrid, const int32_t *qgrid, int n_modes,
                       const double *hw, const double *nph, double sigma, double n_q_norm,
                       int64_t n_ch, const int32_t *ch_i, const int32_t *ch_j,
                       const int8_t *ch_nu, const double *g2, const double *f,
                       const double *lam, double *gf, double *gg2) {
    orc_sys s = make_sys(n_states, state_k, eps, kgrid, qgrid, n_modes, hw, nph, sigma, n_q_norm);
    if (gf) memset(gf, 0, sizeof(double) * (size_t)n_states);
    for (int64_t c = 0; c < n_ch; ++c) {
        int i = ch_i[c], j = ch_j[c], nu = ch_nu[c];
        double a_fi, a_fj, a_g, b_fj, b_fi, b_g;
        term_grads(&s, f, i, j, nu, g2[c], &a_fi, &a_fj, &a_g);   /* T(i,j) feeds I_i */
        term_grads(&s, f, j, i, nu, g2[c], &b_fj, &b_fi, &b_g);   /* T(j,i) feeds I_j */
        if (gf) {
            gf[i] += lam[i] * a_fi + lam[j] * b_fi;
            gf[j] += lam[i] * a_fj + lam[j] * b_fj;
        }
        if (gg2) gg2[c] = lam[i] * a_g + lam[j] * b_g;
    }
}

/*
 * Linearisation of I at (f0, N) for the transport equation: with
 * J = dI/df at f0, the diagonal is J_dd = -1/tau_d and the off-diagonal
 * part is J_dp = W_dp.  Computed by summing the hand-derived partials of
 * every term (the same partials as the reverse mode above):
 *   tau_inv[d] = -sum over terms T(d, .) of dT/df_d
 *   W_ij[c]    = dT(i,j)/df_j   (entry of row i, column j)
 *   W_ji[c]    = dT(j,i)/df_i   (entry of row j, column i)
 */
void orc_transport_coeffs(int n_states, const int32_t *state_k, const double *eps,
                          const int32_t *kgrid, const int32_t *qgrid, int n_modes,
                          const double *hw, const double *nph, double sigma, double n_q_norm,
                          int64_t n_ch, const int32_t *ch_i, const int32_t *ch_j,
                          const int8_t *ch_nu, const double *g2, const double *f0,
                          double *tau_inv, double *W_ij, double *W_ji) {
    orc_sys s = make_sys(n_states, state_k, eps, kgrid, qgrid, n_modes, hw, nph, sigma, n_q_norm);
    memset(tau_inv, 0, sizeof(double) * (size_t)n_states);
    for (int64_t c = 0; c < n_ch; ++c) {
        int i = ch_i[c], j = ch_j[c], nu = ch_nu[c];
        double a_fi, a_fj, a_g, b_fj, b_fi, b_g;
        term_grads(&s, f0, i, j, nu, g2[c], &a_fi, &a_fj, &a_g);
        term_grads(&s, f0, j, i, nu, g2[c], &b_fj, &b_fi, &b_g);
        tau_inv[i] -= a_fi;
        tau_inv[j] -= b_fj;
        W_ij[c] = a_fj;
        W_ji[c] = b_fi;
    }
}

/*
 * In- and out-scattering rates of every state, from the same terms as
 * orc_collision: T(d,p) = In - Out with
 *   Out = P g2 f_d (1 - f_p) [G(e_d - e_p + hw) N + G(e_d - e_p - hw) (N + 1)]
 *   In  = P g2 f_p (1 - f_d) [G(e_d - e_p + hw) (N + 1) + G(e_d - e_p - hw) N]
 * (the gross rates used to judge cancellation near equilibrium).
 */
void orc_collision_inout(int n_states, const int32_t *state_k, const double *eps,
                         const int32_t *kgrid, const int32_t *qgrid, int n_modes,
                         const double *hw, const double *nph, double sigma, double n_q_norm,
                         int64_t n_ch, const int32_t *ch_i, const int32_t *ch_j,
                         const int8_t *ch_nu, const double *g2, const double *f,
                         double *rate_in, double *rate_out) {
    orc_sys s = make_sys(n_states, state_k, eps, kgrid, qgrid, n_modes, hw, nph, sigma, n_q_norm);
    memset(rate_in, 0, sizeof(double) * (size_t)n_states);
    memset(rate_out, 0, sizeof(double) * (size_t)n_states);
    double P = 2.0 * ORC_PI / ORC_HBAR_EV_FS / n_q_norm;
    for (int64_t c = 0; c < n_ch; ++c) {
        for (int side = 0; side < 2; ++side) {
            int d = side ? ch_j[c] : ch_i[c], p = side ? ch_i[c] : ch_j[c], nu = ch_nu[c];
            int q = q_index(&s, d, p);
            double w = hw[(long)q * n_modes + nu], N = nph[(long)q * n_modes + nu];
            double de = eps[d] - eps[p];
            double Ga = gauss(de + w, sigma), Ge = gauss(de - w, sigma);
            rate_out[d] += P * g2[c] * f[d] * (1.0 - f[p]) * (Ga * N + Ge * (N + 1.0));
            rate_in[d] += P * g2[c] * f[p] * (1.0 - f[d]) * (Ga * (N + 1.0) + Ge * N);
        }
    }
}
