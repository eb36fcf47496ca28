/*
 * osc_oracle.c -- CPU FP64 oracle for event-by-event neutrino-oscillation
 * reweighting through constant-density matter (arXiv:1311.7579).
 *
 * TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the CPU
 * baseline timing.  The GPU library never links or calls this file, and
 * this file includes nothing from the GPU library.
 *
 * The computation follows the paper's route in its order:
 *   Sec. 1.1   the PMNS matrix and the vacuum phases m_i^2 L / 2E (Eq. 1);
 *   Sec. 1.1   matter effects on nu_e / anti-nu_e from forward scattering
 *              on electrons (the matter-modified mass matrix);
 *   Sec. 2.1   parameter-only quantities first, then per energy the
 *              eigenvalues of the modified mass matrix from its
 *              characteristic cubic (analytic trigonometric solution),
 *              the transition amplitude, and P = |A|^2 in double
 *              precision;
 *   Sec. 1.1.1 event-by-event reweighting into a binned PDF.
 * It works in the mass basis with full complex 3x3 matrices on purpose:
 * slow and plain, so it can be checked by eye.
 *
 * Built with -ffp-contract=off so that every operation is separately
 * rounded.
 */
#include "osc_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- physical constants (CODATA 2018 / PDG) ---------------------------- */
static const double HBARC_EV_M = 1.973269804e-7;   /* hbar*c in eV*m          */
static const double AVOGADRO   = 6.02214076e23;    /* per mol                 */
static const double GFERMI     = 1.1663787e-5;     /* G_F/(hbar c)^3, GeV^-2  */

double oracle_k_phase(void)
{
    /* m^2 L / (2E):  L[km] -> 1e3 m / (hbar c) eV^-1,  E[GeV] -> 1e9 eV. */
    return 1e3 / (2.0 * 1e9 * HBARC_EV_M);
}

double oracle_k_matter(void)
{
    /* A = 2 sqrt(2) G_F N_e E with N_e = rho * Ye * N_A per cm^3,
     * converted to eV^3 with (hbar c in eV*cm)^3; G_F in eV^-2; E in eV. */
    const double hbarc_cm = HBARC_EV_M * 100.0;
    const double gf_ev = GFERMI * 1e-18;
    return 2.0 * sqrt(2.0) * gf_ev * AVOGADRO * hbarc_cm * hbarc_cm * hbarc_cm * 1e9;
}

/* ---- PMNS matrix, PDG parameterisation (Sec. 1.1) ---------------------- */
static void pmns(const oracle_params* p, int anti, double complex U[3][3])
{
    const double s12 = sqrt(p->sin2_th12), c12 = sqrt(1.0 - p->sin2_th12);
    const double s23 = sqrt(p->sin2_th23), c23 = sqrt(1.0 - p->sin2_th23);
    const double s13 = sqrt(p->sin2_th13), c13 = sqrt(1.0 - p->sin2_th13);
    const double complex eid = cexp(I * p->delta_cp);   /* e^{+i delta} */
    const double complex emid = conj(eid);              /* e^{-i delta} */

    U[0][0] = c12 * c13;
    U[0][1] = s12 * c13;
    U[0][2] = s13 * emid;
    U[1][0] = -s12 * c23 - c12 * s23 * s13 * eid;
    U[1][1] = c12 * c23 - s12 * s23 * s13 * eid;
    U[1][2] = s23 * c13;
    U[2][0] = s12 * s23 - c12 * c23 * s13 * eid;
    U[2][1] = -c12 * s23 - s12 * c23 * s13 * eid;
    U[2][2] = c23 * c13;

    if (anti) {
        for (int a = 0; a < 3; ++a)
            for (int i = 0; i < 3; ++i) U[a][i] = conj(U[a][i]);
    }
}

void oracle_pmns(const oracle_params* p, int anti, double* out)
{
    double complex U[3][3];
    pmns(p, anti, U);
    for (int a = 0; a < 3; ++a)
        for (int i = 0; i < 3; ++i) {
            out[2 * (3 * a + i)] = creal(U[a][i]);
            out[2 * (3 * a + i) + 1] = cimag(U[a][i]);
        }
}

/* squared masses relative to m_1: (0, dm21, dm31), dm31 = dm32 + dm21 */
static void mass_squares(const oracle_params* p, double m2[3])
{
    m2[0] = 0.0;
    m2[1] = p->dm2_21;
    m2[2] = p->dm2_32 + p->dm2_21;
}

/* ---- Eq. (1), corrected: vacuum amplitude ------------------------------ */
double oracle_prob_vacuum(const oracle_params* p, double L_km, double E,
                          int alpha, int beta, int anti)
{
    double complex U[3][3];
    double m2[3];
    pmns(p, anti, U);
    mass_squares(p, m2);
    const double k = oracle_k_phase();
    double complex amp = 0.0;
    for (int i = 0; i < 3; ++i) {
        const double phase = k * m2[i] * L_km / E;
        amp += conj(U[alpha][i]) * U[beta][i] * cexp(-I * phase);
    }
    return creal(amp) * creal(amp) + cimag(amp) * cimag(amp);
}

/* ---- complex 3x3 helpers ------------------------------------------------ */
static void mat_mul(double complex A[3][3], double complex B[3][3],
                    double complex C[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double complex s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[i][k] * B[k][j];
            C[i][j] = s;
        }
}

/* ---- the matter path (Sec. 1.1 matter effects, Sec. 2.1) ---------------- */
/* Evolution operator over L at constant density in the flavour basis,
 * Sf[beta][alpha] = amplitude alpha -> beta. */
static void evolution_flavour(double complex U[3][3], const double m2[3], double A,
                              double L_km, double E, double complex Sf[3][3])
{
    /* Matter-modified mass matrix (2E times the Hamiltonian) in the mass
     * basis: M_ij = m_i^2 delta_ij + A conj(U_ei) U_ej. */
    double complex M[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            M[i][j] = (i == j ? m2[i] : 0.0) + A * conj(U[0][i]) * U[0][j];

    /* Characteristic polynomial  lambda^3 - a lambda^2 + b lambda - c:
     * a = trace, b = sum of principal 2x2 minors, c = determinant. */
    const double a = creal(M[0][0] + M[1][1] + M[2][2]);
    const double b = creal(M[0][0] * M[1][1] - M[0][1] * M[1][0]
                           + M[0][0] * M[2][2] - M[0][2] * M[2][0]
                           + M[1][1] * M[2][2] - M[1][2] * M[2][1]);
    const double c = creal(M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1])
                           - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
                           + M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]));

    /* Analytic (trigonometric) roots of the cubic: with
     * pp = a^2 - 3b and qq = 2a^3 - 9ab + 27c, the roots are
     * a/3 + (2/3) sqrt(pp) cos(theta - 2 pi k / 3),
     * theta = acos(qq / (2 pp^(3/2))) / 3. */
    const double pp = a * a - 3.0 * b;
    const double qq = 2.0 * a * a * a - 9.0 * a * b + 27.0 * c;
    const double sp = sqrt(pp);
    double r = qq / (2.0 * pp * sp);
    if (r > 1.0) r = 1.0;
    if (r < -1.0) r = -1.0;
    const double theta = acos(r) / 3.0;
    double lam[3];
    for (int k = 0; k < 3; ++k)
        lam[k] = a / 3.0 + (2.0 / 3.0) * sp * cos(theta - 2.0 * M_PI * k / 3.0);

    /* Evolution operator over L from the spectral projectors
     * X_k = (M - lam_j)(M - lam_l) / ((lam_k - lam_j)(lam_k - lam_l)):
     * S = sum_k exp(-i kphi lam_k L / E) X_k  (mass basis). */
    const double kphi = oracle_k_phase();
    double complex S[3][3];
    memset(S, 0, sizeof S);
    for (int k = 0; k < 3; ++k) {
        const int j = (k + 1) % 3, l = (k + 2) % 3;
        double complex Mj[3][3], Ml[3][3], X[3][3];
        for (int r0 = 0; r0 < 3; ++r0)
            for (int c0 = 0; c0 < 3; ++c0) {
                Mj[r0][c0] = M[r0][c0] - (r0 == c0 ? lam[j] : 0.0);
                Ml[r0][c0] = M[r0][c0] - (r0 == c0 ? lam[l] : 0.0);
            }
        mat_mul(Mj, Ml, X);
        const double denom = (lam[k] - lam[j]) * (lam[k] - lam[l]);
        const double complex ph = cexp(-I * (kphi * lam[k] * L_km / E));
        for (int r0 = 0; r0 < 3; ++r0)
            for (int c0 = 0; c0 < 3; ++c0) S[r0][c0] += ph * X[r0][c0] / denom;
    }

    /* Back to the flavour basis: S_f = U S U^dagger; amplitude alpha->beta
     * is S_f[beta][alpha]. */
    double complex Ud[3][3], T[3][3];
    for (int r0 = 0; r0 < 3; ++r0)
        for (int c0 = 0; c0 < 3; ++c0) Ud[r0][c0] = conj(U[c0][r0]);
    mat_mul(U, S, T);
    mat_mul(T, Ud, Sf);
}

static double prob_matter(double complex U[3][3], const double m2[3], double A,
                          double L_km, double E, int alpha, int beta)
{
    double complex Sf[3][3];
    evolution_flavour(U, m2, A, L_km, E, Sf);
    const double complex amp = Sf[beta][alpha];
    return creal(amp) * creal(amp) + cimag(amp) * cimag(amp);
}

double oracle_prob(const oracle_params* p, double L_km, double rho, double Ye,
                   double E, int alpha, int beta, int anti)
{
    double complex U[3][3];
    double m2[3];
    pmns(p, anti, U);
    mass_squares(p, m2);
    /* antineutrinos: U -> conj(U) (done in pmns) and A -> -A */
    const double A = (anti ? -1.0 : 1.0) * oracle_k_matter() * Ye * rho * E;
    return prob_matter(U, m2, A, L_km, E, alpha, beta);
}

double oracle_prob_layered(const oracle_params* p, int32_t n_layers, const double* L_km,
                           const double* rho, const double* Ye, double E,
                           int alpha, int beta, int anti)
{
    double complex U[3][3];
    double m2[3];
    pmns(p, anti, U);
    mass_squares(p, m2);
    /* S = S_{n-1} ... S_0, the first layer crossed on the right */
    double complex S[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) S[i][j] = (i == j) ? 1.0 : 0.0;
    for (int32_t k = 0; k < n_layers; ++k) {
        const double A = (anti ? -1.0 : 1.0) * oracle_k_matter() * Ye[k] * rho[k] * E;
        double complex Sk[3][3], T[3][3];
        evolution_flavour(U, m2, A, L_km[k], E, Sk);
        mat_mul(Sk, S, T);
        memcpy(S, T, sizeof S);
    }
    const double complex amp = S[beta][alpha];
    return creal(amp) * creal(amp) + cimag(amp) * cimag(amp);
}

void oracle_prob_layered_batch(const oracle_params* p, int32_t n_layers, const double* L_km,
                               const double* rho, const double* Ye, int64_t n,
                               const double* E, const uint8_t* flags, double* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const uint8_t f = flags[i];
        const int alpha = f & 3, beta = (f >> 2) & 3, anti = (f >> 4) & 1;
        out[i] = (alpha > 2 || beta > 2 || (f >> 5) != 0)
                     ? NAN
                     : oracle_prob_layered(p, n_layers, L_km, rho, Ye, E[i], alpha, beta, anti);
    }
}

static double prob_from_flags(const oracle_params* p, double L_km, double rho,
                              double Ye, double E, uint8_t f)
{
    const int alpha = f & 3, beta = (f >> 2) & 3, anti = (f >> 4) & 1;
    if (alpha > 2 || beta > 2 || (f >> 5) != 0) return NAN;
    return oracle_prob(p, L_km, rho, Ye, E, alpha, beta, anti);
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_prob_batch(const oracle_params* p, double L_km, double rho, double Ye,
                      int64_t n, const double* e_true, const uint8_t* flags,
                      double* p_out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        p_out[i] = prob_from_flags(p, L_km, rho, Ye, e_true[i], flags[i]);
    return oracle_num_threads();
}

/* ---- binning and the deterministic histogram (Sec. 1.1.1) -------------- */
int32_t oracle_bin_index(double x, double lo, double hi, int32_t nbins)
{
    const double wb = (hi - lo) / (double)nbins;
    const double q = (x - lo) / wb;
    if (q < 0.0) return nbins;                   /* underflow */
    if (!(q < (double)nbins)) return nbins + 1;  /* overflow, NaN */
    return (int32_t)floor(q);
}

int32_t oracle_bin_index_scaled(double x, double e_scale, double lo, double hi, int32_t nbins)
{
    const double scale = 1.0 + e_scale;
    const double xs = x * scale;
    return oracle_bin_index(xs, lo, hi, nbins);
}

/* the rule of oracle_bin_index_scaled applied to x[0..n) */
void oracle_bin_indices_scaled(int64_t n, const double* x, double e_scale, double lo, double hi,
                               int32_t nbins, int32_t* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = oracle_bin_index_scaled(x[i], e_scale, lo, hi, nbins);
}

/* complete binary tree sum of v[0..npow2), entries at or beyond nreal
 * counting as +0.0; left subtree + right subtree at every node */
static double tree_sum(const double* v, int64_t nreal, int64_t npow2)
{
    if (npow2 == 1) return nreal > 0 ? v[0] : 0.0;
    const int64_t half = npow2 / 2;
    const int64_t nl = nreal < half ? nreal : half;
    const int64_t nr = nreal > half ? nreal - half : 0;
    const double left = tree_sum(v, nl, half);
    const double right = tree_sum(v + half, nr, half);
    return left + right;
}

void oracle_hist_contract(const double* c, const int32_t* bin, int64_t n,
                          int32_t nbt, int32_t W, int32_t K, int32_t A, double* out)
{
    const int64_t T = (int64_t)W * K;
    const int64_t ntiles = (n + T - 1) / T;
    int64_t p2 = 1;
    while (p2 < ntiles) p2 *= 2;

    /* per-bin tile results, bin-major */
    double* tiles = (double*)calloc((size_t)(ntiles > 0 ? ntiles : 1) * nbt, sizeof(double));
    double* acc = (double*)malloc((size_t)A * nbt * sizeof(double));
    double* col = (double*)malloc((size_t)A * sizeof(double));

    for (int64_t t = 0; t < ntiles; ++t) {
        /* every accumulator starts from +0.0 in every bin */
        for (int64_t q = 0; q < (int64_t)A * nbt; ++q) acc[q] = 0.0;
        /* event slot m after event slot m; within a slot, ascending lane,
         * lane l adding into accumulator l mod A */
        for (int32_t m = 0; m < K; ++m)
            for (int32_t l = 0; l < W; ++l) {
                const int64_t i = t * T + (int64_t)m * W + l;
                if (i >= n) continue;
                acc[(int64_t)bin[i] * A + l % A] += c[i];
            }
        for (int32_t b = 0; b < nbt; ++b) {
            for (int32_t a = 0; a < A; ++a) col[a] = acc[(int64_t)b * A + a];
            tiles[(int64_t)b * ntiles + t] = tree_sum(col, A, A);
        }
    }
    for (int32_t b = 0; b < nbt; ++b)
        out[b] = ntiles > 0 ? tree_sum(tiles + (int64_t)b * ntiles, ntiles, p2) : 0.0;

    free(col);
    free(acc);
    free(tiles);
}

void oracle_template(int64_t n, const double* e_true, const uint8_t* flags,
                     const double* weight, const double* e_reco,
                     int32_t nt, double lo_t, double hi_t,
                     int32_t nr, double lo_r, double hi_r, double e_scale,
                     double* T, int64_t* n_used)
{
    const int64_t K = 18 * (int64_t)nt;
    for (int64_t q = 0; q < (int64_t)(nr + 2) * K; ++q) T[q] = 0.0;
    int64_t used = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int alpha = flags[i] & 3, beta = (flags[i] >> 2) & 3, anti = (flags[i] >> 4) & 1;
        if (flags[i] >= 32 || alpha == 3 || beta == 3) continue;
        const int32_t t = oracle_bin_index(e_true[i], lo_t, hi_t, nt);
        if (t >= nt) continue;   /* underflow (nt) or overflow (nt + 1) */
        const int32_t r = oracle_bin_index_scaled(e_reco[i], e_scale, lo_r, hi_r, nr);
        const int64_t c = alpha + 3 * beta + 9 * anti;
        T[(int64_t)r * K + c * nt + t] += weight[i];
        ++used;
    }
    if (n_used) *n_used = used;
}

double oracle_bin_centre(double lo, double hi, int32_t nt, int32_t t)
{
    const double wb = (hi - lo) / (double)nt;
    const double off = ((double)t + 0.5) * wb;
    return lo + off;
}

void oracle_centre_probs(const oracle_params* p, double L_km, double rho, double Ye,
                         int32_t nt, double lo_t, double hi_t, double* P)
{
    for (int c = 0; c < 18; ++c) {
        const int alpha = c % 3, beta = (c / 3) % 3, anti = c / 9;
        for (int32_t t = 0; t < nt; ++t)
            P[(int64_t)c * nt + t] = oracle_prob(p, L_km, rho, Ye, oracle_bin_centre(lo_t, hi_t, nt, t),
                                                alpha, beta, anti);
    }
}

void oracle_bincentre_contract(const double* T, const double* P, int32_t K, int32_t nrt,
                               double* hist)
{
    double lanes[64];
    for (int32_t r = 0; r < nrt; ++r) {
        for (int l = 0; l < 64; ++l) lanes[l] = 0.0;
        for (int32_t k = 0; k < K; ++k) {
            const double term = T[(int64_t)r * K + k] * P[k];
            lanes[k % 64] += term;
        }
        hist[r] = tree_sum(lanes, 64, 64);
    }
}

double oracle_poisson_nll(const double* mu, const double* data, int32_t nbins)
{
    double s = 0.0;
    for (int32_t b = 0; b < nbins; ++b) {
        const double m = mu[b], d = data[b];
        double term;
        if (m == 0.0)
            term = d == 0.0 ? 0.0 : INFINITY;
        else
            term = m - d * log(m) + lgamma(d + 1.0);
        s += term;
    }
    return 2.0 * s;
}

int oracle_fill_pdf(const oracle_params* p, double L_km, double rho, double Ye,
                    int64_t n, const double* e_true, const uint8_t* flags,
                    const double* weight, const double* e_reco,
                    int32_t nbins, double lo, double hi, double e_scale, int32_t W, int32_t K,
                    int32_t A, double* hist_out, double* p_out)
{
    double* prob = p_out ? p_out : (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double* c = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    int32_t* b = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    const int threads = oracle_prob_batch(p, L_km, rho, Ye, n, e_true, flags, prob);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        c[i] = weight[i] * prob[i];
        b[i] = oracle_bin_index_scaled(e_reco[i], e_scale, lo, hi, nbins);
    }
    oracle_hist_contract(c, b, n, nbins + 2, W, K, A, hist_out);
    free(b);
    free(c);
    if (!p_out) free(prob);
    return threads;
}
