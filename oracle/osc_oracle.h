/*
 * osc_oracle.h -- CPU FP64 oracle for event-by-event oscillation reweighting.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * check and the CPU-baseline timing can compare the GPU library against a
 * plain, slow, obviously correct implementation written from the paper
 * (arXiv:1311.7579, "Accelerated Event-by-Event Neutrino Oscillation
 * Reweighting with Matter Effects on a GPU").  Product code never links,
 * loads or calls it.  It shares no source with the GPU library.
 *
 * Conventions (identical meaning to the product's public header, written
 * independently):
 *   flavour index 0 = e, 1 = mu, 2 = tau;
 *   energies in GeV, baseline in km, mass splittings in eV^2,
 *   density in g/cm^3, Ye = electrons per nucleon.
 *   Event flag byte: bits 0-1 initial flavour alpha, bits 2-3 final flavour
 *   beta, bit 4 antineutrino.
 *   Histogram layout: nbins regular bins, then underflow, then overflow.
 */
#ifndef OSC_ORACLE_H
#define OSC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The six oscillation parameters of Table 1 (sin^2 of the three mixing
 * angles, the two mass splittings, the CP phase in radians). */
typedef struct {
    double sin2_th12, sin2_th23, sin2_th13;
    double dm2_32, dm2_21;
    double delta_cp;
} oracle_params;

/* Phase constant: the vacuum phase m^2 L / (2E) in natural units equals
 * oracle_k_phase() * m^2[eV^2] * L[km] / E[GeV]. */
double oracle_k_phase(void);

/* Matter constant: 2 sqrt(2) G_F N_e E equals
 * oracle_k_matter() * Ye * rho[g/cm^3] * E[GeV]  (eV^2). */
double oracle_k_matter(void);

/* PMNS matrix (PDG parameterisation) as interleaved re/im, row = flavour,
 * column = mass state: out[2*(3*a+i)] = Re U_ai, out[2*(3*a+i)+1] = Im U_ai.
 * anti != 0 returns the complex conjugate (antineutrino rule). */
void oracle_pmns(const oracle_params* p, int anti, double* out);

/* Sec. 1.1, Eq. (1) in corrected form: vacuum transition probability
 * P(alpha -> beta) = |sum_i conj(U_alpha i) U_beta i exp(-i k m_i^2 L/E)|^2. */
double oracle_prob_vacuum(const oracle_params* p, double L_km, double E,
                          int alpha, int beta, int anti);

/* Sec. 1.1 and 2.1: probability through constant-density matter via the
 * matter-modified mass matrix, its analytic characteristic-cubic
 * eigenvalues and the projector expansion of the evolution operator.
 * rho may be negative (test hook: flips the sign of the matter term
 * independently of the antineutrino flag). */
double oracle_prob(const oracle_params* p, double L_km, double rho, double Ye,
                   double E, int alpha, int beta, int anti);

/* P(alpha -> beta) through n_layers layers of constant density (lengths
 * L_km[k], densities rho[k], electron fractions Ye[k]; layer 0 crossed
 * first): the amplitude is element (beta, alpha) of the product
 * S_{n-1} ... S_1 S_0 of the layers' flavour-basis evolution operators,
 * each computed as in oracle_prob.  Not in the paper (its path has one
 * density); the layered path is the extension its CPU library makes. */
double oracle_prob_layered(const oracle_params* p, int32_t n_layers, const double* L_km,
                           const double* rho, const double* Ye, double E,
                           int alpha, int beta, int anti);

/* oracle_prob_layered over events described by flag bytes (NaN for an
 * invalid flag byte), OpenMP. */
void oracle_prob_layered_batch(const oracle_params* p, int32_t n_layers, const double* L_km,
                               const double* rho, const double* Ye, int64_t n,
                               const double* E, const uint8_t* flags, double* out);

/* Same as oracle_prob for arrays of events described by flag bytes.
 * OpenMP-parallel over events; returns the thread count used. */
int oracle_prob_batch(const oracle_params* p, double L_km, double rho, double Ye,
                      int64_t n, const double* e_true, const uint8_t* flags,
                      double* p_out);

/* Bin index of one reconstructed energy: q = (x - lo) / wb with
 * wb = (hi - lo) / nbins, both IEEE FP64 operations; q < 0 -> nbins
 * (underflow), q >= nbins or NaN -> nbins + 1 (overflow), else floor(q). */
int32_t oracle_bin_index(double x, double lo, double hi, int32_t nbins);

/* Bin index of a reconstructed energy under a relative energy-scale shift
 * (the systematic of Sec. 1.1.1): the bin of x * (1 + e_scale), both FP64
 * operations, by the rule above. */
int32_t oracle_bin_index_scaled(double x, double e_scale, double lo, double hi, int32_t nbins);

/* oracle_bin_index_scaled of every x[i], i < n, into out[i]. */
void oracle_bin_indices_scaled(int64_t n, const double* x, double e_scale, double lo, double hi,
                               int32_t nbins, int32_t* out);

/* Deterministic histogram of contributions c[i] into bin[i] (values in
 * [0, nbt)) following the tile reduction contract with tile width W lanes,
 * K events per lane and A accumulators per bin (powers of two, A divides W):
 *   tile t holds events t*W*K .. t*W*K + W*K - 1; lane l of the tile takes
 *   events t*W*K + m*W + l for m = 0..K-1;
 *   lane l adds into accumulator l mod A of the event's bin; every
 *   accumulator starts from +0.0 and receives its additions in ascending
 *   m and, within one m, in ascending l;
 *   for each bin, the A accumulators of a tile are added by the complete
 *   binary tree over accumulator index (adjacent pairs first);
 *   for each bin, the tile results are added by the complete binary tree
 *   over tile index, padded with +0.0 to a power of two.
 * out has nbt entries. */
void oracle_hist_contract(const double* c, const int32_t* bin, int64_t n,
                          int32_t nbt, int32_t W, int32_t K, int32_t A, double* out);

/* Plain reweight + binned PDF (Sec. 1.1.1): P per event, contribution
 * c = w * P (separately rounded), bin of e_reco, histogram by the tile
 * contract above, reconstructed energies scaled by (1 + e_scale) before
 * binning.  hist_out has nbins + 2 entries; p_out may be NULL. */
int oracle_fill_pdf(const oracle_params* p, double L_km, double rho, double Ye,
                    int64_t n, const double* e_true, const uint8_t* flags,
                    const double* weight, const double* e_reco,
                    int32_t nbins, double lo, double hi, double e_scale, int32_t W, int32_t K,
                    int32_t A, double* hist_out, double* p_out);

/* ---- Bin-centre reweighting (Sec. 1.1.1): the approximation that the
 * event-by-event method replaces.  The sample is reduced once to a
 * migration template; a parameter set is then applied through P evaluated
 * at the centre of each true-energy bin.
 *
 * Channel c = alpha + 3 beta + 9 anti (18 channels).  True bin t of E by
 * oracle_bin_index(E, lo_t, hi_t, nt) (events outside [0, nt), and events
 * with an invalid flag byte, are left out); reconstructed bin r by
 * oracle_bin_index_scaled(e_reco, e_scale, lo_r, hi_r, nr), r in
 * [0, nr + 2).  Template layout T[r][c][t] (reco-bin major): the weights of
 * the cell's events summed in ascending event order from +0.0.  *n_used
 * receives the number of events in the template. */
void oracle_template(int64_t n, const double* e_true, const uint8_t* flags,
                     const double* weight, const double* e_reco,
                     int32_t nt, double lo_t, double hi_t,
                     int32_t nr, double lo_r, double hi_r, double e_scale,
                     double* T, int64_t* n_used);

/* Centre of true bin t: lo + (t + 1/2) * ((hi - lo) / nt), FP64, the
 * width and each operation rounded separately. */
double oracle_bin_centre(double lo, double hi, int32_t nt, int32_t t);

/* P_c(E_t) for the 18 channels at every true-bin centre, layout P[c][t]. */
void oracle_centre_probs(const oracle_params* p, double L_km, double rho, double Ye,
                         int32_t nt, double lo_t, double hi_t, double* P);

/* hist[r] = sum over k = c nt + t of fl(T[r][k] * P[k]) for r in [0, nrt):
 * term k goes to lane k mod 64, each lane adds its terms in ascending k
 * from +0.0, and the 64 lane sums meet in the complete binary tree over
 * lane index (adjacent pairs first). */
void oracle_bincentre_contract(const double* T, const double* P, int32_t K, int32_t nrt,
                               double* hist);

/* Sec. 2.2, Eq. (2), read as a product over the regular bins of Poisson
 * probabilities of the observed counts d_b given the expectations mu_b:
 * -2 ln L = 2 sum_b (mu_b - d_b ln mu_b + ln d_b!)  (ln d! = lgamma(d + 1)).
 * A bin with mu_b = 0 adds 0 when d_b = 0 and +infinity otherwise. */
double oracle_poisson_nll(const double* mu, const double* data, int32_t nbins);

/* OpenMP thread count the batch functions use, and a setter (n > 0). */
int oracle_num_threads(void);
void oracle_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
