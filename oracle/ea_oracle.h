/*
 * ea_oracle.h -- plain CPU oracle for checkerboard Metropolis ageing runs of
 * the 3D +-J Edwards-Anderson model (Manssen & Hartmann, "Ageing at the
 * Spin-Glass/Ferromagnet Transition: Monte Carlo Simulation using GPUs").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header or table with the GPU
 * library.
 *
 * Representation: spins S = +-1 and couplings J = +-1 as int8, one per site
 * (one per bond), canonical site index s = x + L*(y + L*z), bond J[s][d]
 * couples s and s + e_d (periodic), d = 0,1,2 for x,y,z ("left/up" bonds,
 * Sec. III).  The coupling array is laid out [s][d] (index 3*s + d).
 *
 * Conventions fixed here (the paper leaves them open; each is listed with its
 * reading in the design notes):
 *   - p is the probability of an antiferromagnetic bond, P(J = -1) = p.
 *   - colour c(s) = (x+y+z) & 1, half index h(s) = (x>>1) + (L/2)(y + L z).
 *   - sweep t (0-based) is: replica r updates colour r, then colour 1-r.
 *   - random words: Philox4x32-10, key = (seed lo, seed hi), counter =
 *     (aux, h>>2, tag<<8 | colour<<1 | replica, sample), word h & 3, where aux
 *     is the sweep index (tag 0), the bond direction (tag 1) or 0 (tag 2).
 *   - shared noise (asynchronous multispin coding, Sec. III): a run switched
 *     by eao_share_noise draws its Metropolis words with tag 3 and counter
 *     word 3 = the shared id instead of its sample, so every run with the same
 *     seed and id uses the same word for the same (sweep, colour, replica,
 *     site); its couplings and start keep the sample's own keys.
 *   - acceptance of dE = 4k > 0 iff u < thr_k, thr_k = floor(exp(-4k/T) 2^32)
 *     (clamped to 2^32-1; 0 at T = 0).  dE <= 0 is always accepted.
 */
#ifndef EA_ORACLE_H
#define EA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Random-word tags (third counter word, bits 8 and up). */
enum { EAO_TAG_METRO = 0, EAO_TAG_BOND = 1, EAO_TAG_INIT = 2, EAO_TAG_SHARED = 3 };

/* Philox4x32-10 block: out = Philox(key, ctr).  Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11. */
void eao_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The 32-bit random word of one site under the keying above. */
uint32_t eao_site_word(uint64_t seed, uint32_t sample, uint32_t tag, uint32_t aux,
                       int colour, int replica, uint64_t h);

/* Acceptance thresholds thr[k-1] for dE = 4k, k = 1..3 (eq. 9). */
void eao_thresholds(double T, uint32_t thr[3]);

/* Colour and half index of canonical site s. */
int eao_colour(int L, int64_t s);
int64_t eao_half_index(int L, int64_t s);

/* Energy H = -sum_<ij> J_ij S_i S_j over the 3N stored bonds (eq. 1). */
int64_t eao_energy(int L, const int8_t *S, const int8_t *J);
/* Local energy change of flipping site s: dE = 2 sum_j J_ij S_i S_j (eq. 9). */
int eao_delta_e(int L, const int8_t *S, const int8_t *J, int64_t s);

typedef struct eao_sim eao_sim;

/* Observables at the current time (all integer sums over the N sites):
 *   unsat[r]      number of unsatisfied bonds of replica r; E_r = 2 unsat - 3N
 *   mag[r]        sum_s S_r(s)
 *   overlap       sum_s S_0(s) S_1(s)                         (eq. 2, times N)
 *   autocorr[r*n_slots + k]  sum_s S_r(s,t) S_r(s,tw_k)        (eq. 7, times N);
 *                            0 for a slot that was never taken
 *   c4[d*(L/2+1) + rho]      sum_s q(s) q(s + rho e_d), q = S_0 S_1 (eq. 3, times N)
 * The caller owns the arrays (autocorr: 2*n_slots, c4: 3*(L/2+1)). */
typedef struct {
    uint64_t t;
    int64_t unsat[2];
    int64_t mag[2];
    int64_t overlap;
    int64_t *autocorr;
    int64_t *c4;
} eao_obs;

/* Create a run: couplings and both replicas' initial spins from the keyed
 * words (quench from infinite temperature, Sec. II).  Returns NULL on bad
 * arguments: L < 2 or odd, p outside [0,1], T < 0 or not finite,
 * n_slots < 0. */
eao_sim *eao_create(int L, double p, double T, uint64_t seed, uint32_t sample, int n_slots);
void eao_destroy(eao_sim *sim);

int eao_L(const eao_sim *sim);
uint64_t eao_time(const eao_sim *sim);
void eao_set_time(eao_sim *sim, uint64_t t);
/* From now on draw the Metropolis words from the shared stream `id` (see the
 * conventions above): the samples that one multispin word holds in the
 * paper's Sec. III all follow one random number per site and sweep. */
void eao_share_noise(eao_sim *sim, uint32_t id);

/* Advance both replicas by n sweeps. */
void eao_sweep(eao_sim *sim, uint64_t n);
/* One checkerboard half-step (half = 0 or 1) of sweep index eao_time(); the
 * time advances after half 1.  Exposed for the update-order tests. */
void eao_half_step(eao_sim *sim, int half);
/* As eao_half_step, but visiting the sites of the active colour in the
 * order given by perm (a permutation of 0..N/2-1 over half indices). */
void eao_half_step_order(eao_sim *sim, int half, const int64_t *perm);

/* Store the current spins as the reference configuration of slot k. */
int eao_snapshot(eao_sim *sim, int slot);
uint64_t eao_snapshot_time(const eao_sim *sim, int slot);

void eao_measure(const eao_sim *sim, eao_obs *out);

/* Full-vector four-point correlation by distance shells (eq. 3 with every
 * displacement r, not only the axes): out[k] = sum over all r in Z_L^3 whose
 * minimum-image squared length |r|^2 = sum_d min(r_d, L - r_d)^2 equals k of
 * sum_s q(s) q(s + r), q = S_0 S_1, for k = 0 .. n_shells - 1 (shells beyond
 * are not reported).  Direct double sum, O(N^2). */
void eao_c4_shells(const eao_sim *sim, int n_shells, int64_t *out);

void eao_get_spins(const eao_sim *sim, int r, int8_t *S);
void eao_set_spins(eao_sim *sim, int r, const int8_t *S);
void eao_get_bonds(const eao_sim *sim, int8_t *J);
void eao_set_bonds(eao_sim *sim, const int8_t *J);

#ifdef __cplusplus
}
#endif
#endif
