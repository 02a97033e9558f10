/*
 * ea_oracle.c -- plain CPU oracle (test infrastructure only; see ea_oracle.h).
 *
 * Written for clarity, not speed: int8 spins and couplings, one site at a
 * time, every observable summed from its definition.  Each function names
 * the part of the paper it follows.
 */
#include "ea_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11): a 10-round keyed bijection on four
 * 32-bit words.  Each round multiplies words 0 and 2 by fixed odd constants,
 * takes the 64-bit products apart, and mixes the high halves with words 1 and
 * 3 and the round key; the key is bumped by two Weyl constants between
 * rounds. */

#define EAO_PHILOX_M0 0xD2511F53u
#define EAO_PHILOX_M1 0xCD9E8D57u
#define EAO_PHILOX_W0 0x9E3779B9u
#define EAO_PHILOX_W1 0xBB67AE85u

static void mul_hi_lo(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo)
{
    uint64_t prod = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(prod >> 32);
    *lo = (uint32_t)prod;
}

void eao_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint32_t hi0, lo0, hi1, lo1;
        mul_hi_lo(EAO_PHILOX_M0, x[0], &hi0, &lo0);
        mul_hi_lo(EAO_PHILOX_M1, x[2], &hi1, &lo1);
        uint32_t y0 = hi1 ^ x[1] ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x[3] ^ k1;
        uint32_t y3 = lo0;
        x[0] = y0; x[1] = y1; x[2] = y2; x[3] = y3;
        k0 += EAO_PHILOX_W0;
        k1 += EAO_PHILOX_W1;
    }
    out[0] = x[0]; out[1] = x[1]; out[2] = x[2]; out[3] = x[3];
}

/* The keying of every random word the method draws.  The paper's generator
 * (a 1024-bit Xorshift shared across samples, Sec. III) is replaced by a
 * counter-based one so that each (seed, sample, replica, sweep, site) has its
 * own word, independent of how the work is laid out. */
uint32_t eao_site_word(uint64_t seed, uint32_t sample, uint32_t tag, uint32_t aux,
                       int colour, int replica, uint64_t h)
{
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t ctr[4];
    ctr[0] = aux;
    ctr[1] = (uint32_t)(h >> 2);
    ctr[2] = (tag << 8) | ((uint32_t)colour << 1) | (uint32_t)replica;
    ctr[3] = sample;
    uint32_t out[4];
    eao_philox4x32_10(ctr, key, out);
    return out[h & 3];
}

/* Eq. (9): p_accept = min(1, exp(-dE/T)), dE = 2 sum_j J_ij S_i S_j.  On the
 * cubic lattice dE is one of 0, +-4, +-8, +-12, so three thresholds suffice:
 * a uniform 32-bit word u accepts dE = 4k > 0 iff u < floor(exp(-4k/T) 2^32).
 * At T = 0 no uphill move is accepted. */
void eao_thresholds(double T, uint32_t thr[3])
{
    for (int k = 1; k <= 3; ++k) {
        if (!(T > 0.0)) {
            thr[k - 1] = 0;
            continue;
        }
        double a = exp(-4.0 * (double)k / T);
        double scaled = floor(a * 4294967296.0);
        uint64_t v = (uint64_t)scaled;
        if (v > 0xffffffffull) v = 0xffffffffull;
        thr[k - 1] = (uint32_t)v;
    }
}

/* ------------------------------------------------------------------------ */
/* Lattice geometry (Sec. II): N = L^3 sites, periodic in all directions. */

static int64_t site_of(int L, int x, int y, int z)
{
    x = ((x % L) + L) % L;
    y = ((y % L) + L) % L;
    z = ((z % L) + L) % L;
    return (int64_t)x + (int64_t)L * ((int64_t)y + (int64_t)L * z);
}

static void coords_of(int L, int64_t s, int *x, int *y, int *z)
{
    *x = (int)(s % L);
    *y = (int)((s / L) % L);
    *z = (int)(s / ((int64_t)L * L));
}

int eao_colour(int L, int64_t s)
{
    int x, y, z;
    coords_of(L, s, &x, &y, &z);
    return (x + y + z) & 1;
}

int64_t eao_half_index(int L, int64_t s)
{
    int x, y, z;
    coords_of(L, s, &x, &y, &z);
    return (int64_t)(x >> 1) + (int64_t)(L / 2) * ((int64_t)y + (int64_t)L * z);
}

/* Eq. (1): H = -sum over nearest-neighbour pairs of J_ij S_i S_j.  Each site
 * carries the bonds to its +x, +y and +z neighbours, so summing those 3N bonds
 * counts every pair once. */
int64_t eao_energy(int L, const int8_t *S, const int8_t *J)
{
    int64_t N = (int64_t)L * L * L;
    int64_t H = 0;
    for (int64_t s = 0; s < N; ++s) {
        int x, y, z;
        coords_of(L, s, &x, &y, &z);
        int64_t nb[3] = {site_of(L, x + 1, y, z), site_of(L, x, y + 1, z),
                         site_of(L, x, y, z + 1)};
        for (int d = 0; d < 3; ++d)
            H -= (int64_t)J[3 * s + d] * S[s] * S[nb[d]];
    }
    return H;
}

/* Eq. (9): the energy change of flipping S_i is 2 S_i sum_j J_ij S_j over the
 * six neighbours; the bond to the -d neighbour is the one stored there. */
int eao_delta_e(int L, const int8_t *S, const int8_t *J, int64_t s)
{
    int x, y, z;
    coords_of(L, s, &x, &y, &z);
    int field = 0;
    for (int d = 0; d < 3; ++d) {
        int dx = (d == 0), dy = (d == 1), dz = (d == 2);
        int64_t up = site_of(L, x + dx, y + dy, z + dz);
        int64_t down = site_of(L, x - dx, y - dy, z - dz);
        field += J[3 * s + d] * S[up];
        field += J[3 * down + d] * S[down];
    }
    return 2 * S[s] * field;
}

/* ------------------------------------------------------------------------ */

struct eao_sim {
    int L;
    int64_t N;
    double T;
    uint64_t seed;
    uint32_t sample;
    uint32_t metro_tag;    /* tag and counter word 3 of the Metropolis words */
    uint32_t metro_id;
    uint32_t thr[3];
    uint64_t t;
    int n_slots;
    int8_t *J;          /* [N][3] */
    int8_t *S[2];       /* [N] per replica */
    int8_t *snap;       /* [n_slots][2][N] */
    uint64_t *snap_t;   /* [n_slots] */
};

int eao_L(const eao_sim *sim) { return sim->L; }
uint64_t eao_time(const eao_sim *sim) { return sim->t; }
void eao_set_time(eao_sim *sim, uint64_t t) { sim->t = t; }

/* Sec. III: in asynchronous multispin coding one random number serves the
 * same site of every sample packed in the word.  Only the Metropolis words
 * change; each sample keeps its own couplings and start. */
void eao_share_noise(eao_sim *sim, uint32_t id)
{
    sim->metro_tag = EAO_TAG_SHARED;
    sim->metro_id = id;
}

/* Sec. II: couplings drawn i.i.d. per bond with P(J = -1) = p; both replicas
 * start from independent uniformly random spins (quench from T = infinity);
 * the two replicas share the couplings. */
eao_sim *eao_create(int L, double p, double T, uint64_t seed, uint32_t sample, int n_slots)
{
    if (L < 2 || (L & 1)) return NULL;
    if (!(p >= 0.0 && p <= 1.0)) return NULL;
    if (!(T >= 0.0) || isinf(T)) return NULL;
    if (n_slots < 0) return NULL;

    eao_sim *sim = (eao_sim *)calloc(1, sizeof(eao_sim));
    if (!sim) return NULL;
    sim->L = L;
    sim->N = (int64_t)L * L * L;
    sim->T = T;
    sim->seed = seed;
    sim->sample = sample;
    sim->metro_tag = EAO_TAG_METRO;
    sim->metro_id = sample;
    sim->t = 0;
    sim->n_slots = n_slots;
    eao_thresholds(T, sim->thr);

    int64_t N = sim->N;
    sim->J = (int8_t *)malloc((size_t)(3 * N));
    sim->S[0] = (int8_t *)malloc((size_t)N);
    sim->S[1] = (int8_t *)malloc((size_t)N);
    sim->snap = (int8_t *)calloc((size_t)(n_slots > 0 ? n_slots : 1) * 2 * (size_t)N, 1);
    sim->snap_t = (uint64_t *)calloc((size_t)(n_slots > 0 ? n_slots : 1), sizeof(uint64_t));
    if (!sim->J || !sim->S[0] || !sim->S[1] || !sim->snap || !sim->snap_t) {
        eao_destroy(sim);
        return NULL;
    }

    /* P(J = -1) = p: the bond is antiferromagnetic iff its word is below
     * p * 2^32, compared in 64 bits so that p = 1 makes every bond -1. */
    uint64_t pcut = (uint64_t)floor(ldexp(p, 32));
    for (int64_t s = 0; s < N; ++s) {
        int c = eao_colour(L, s);
        int64_t h = eao_half_index(L, s);
        for (int d = 0; d < 3; ++d) {
            uint32_t u = eao_site_word(seed, sample, EAO_TAG_BOND, (uint32_t)d, c, 0, (uint64_t)h);
            sim->J[3 * s + d] = ((uint64_t)u < pcut) ? (int8_t)-1 : (int8_t)1;
        }
    }
    /* Random initial spins: S = -1 iff the top bit of the word is set. */
    for (int r = 0; r < 2; ++r) {
        for (int64_t s = 0; s < N; ++s) {
            int c = eao_colour(L, s);
            int64_t h = eao_half_index(L, s);
            uint32_t u = eao_site_word(seed, sample, EAO_TAG_INIT, 0, c, r, (uint64_t)h);
            sim->S[r][s] = (u >> 31) ? (int8_t)-1 : (int8_t)1;
        }
    }
    return sim;
}

void eao_destroy(eao_sim *sim)
{
    if (!sim) return;
    free(sim->J);
    free(sim->S[0]);
    free(sim->S[1]);
    free(sim->snap);
    free(sim->snap_t);
    free(sim);
}

/* Metropolis update of one site (eq. 9): downhill and neutral moves are
 * always taken; an uphill move dE = 4k is taken iff the site's word for this
 * sweep and colour is below thr_k. */
static void update_site(eao_sim *sim, int r, int colour, int64_t s)
{
    int8_t *S = sim->S[r];
    int dE = eao_delta_e(sim->L, S, sim->J, s);
    int flip;
    if (dE <= 0) {
        flip = 1;
    } else {
        int k = dE / 4;
        uint32_t u = eao_site_word(sim->seed, sim->metro_id, sim->metro_tag, (uint32_t)sim->t,
                                   colour, r, (uint64_t)eao_half_index(sim->L, s));
        flip = u < sim->thr[k - 1];
    }
    if (flip) S[s] = (int8_t)-S[s];
}

/* Checkerboard schedule (Sec. III): a sweep is two half-steps, each updating
 * one sub-lattice given the other.  With the interlaced two-replica layout of
 * Fig. 1, replica r updates colour r in the first half-step and colour 1-r in
 * the second. */
void eao_half_step(eao_sim *sim, int half)
{
    for (int r = 0; r < 2; ++r) {
        int colour = r ^ half;
        for (int64_t s = 0; s < sim->N; ++s)
            if (eao_colour(sim->L, s) == colour) update_site(sim, r, colour, s);
    }
    if (half == 1) sim->t += 1;
}

void eao_half_step_order(eao_sim *sim, int half, const int64_t *perm)
{
    int L = sim->L;
    int64_t half_n = sim->N / 2;
    /* map (colour, half index) back to the canonical site */
    int64_t *site_of_h[2];
    site_of_h[0] = (int64_t *)malloc((size_t)half_n * sizeof(int64_t));
    site_of_h[1] = (int64_t *)malloc((size_t)half_n * sizeof(int64_t));
    for (int64_t s = 0; s < sim->N; ++s)
        site_of_h[eao_colour(L, s)][eao_half_index(L, s)] = s;
    for (int r = 0; r < 2; ++r) {
        int colour = r ^ half;
        for (int64_t i = 0; i < half_n; ++i) update_site(sim, r, colour, site_of_h[colour][perm[i]]);
    }
    free(site_of_h[0]);
    free(site_of_h[1]);
    if (half == 1) sim->t += 1;
}

void eao_sweep(eao_sim *sim, uint64_t n)
{
    for (uint64_t i = 0; i < n; ++i) {
        eao_half_step(sim, 0);
        eao_half_step(sim, 1);
    }
}

int eao_snapshot(eao_sim *sim, int slot)
{
    if (slot < 0 || slot >= sim->n_slots) return -1;
    int64_t N = sim->N;
    memcpy(sim->snap + ((size_t)slot * 2 + 0) * (size_t)N, sim->S[0], (size_t)N);
    memcpy(sim->snap + ((size_t)slot * 2 + 1) * (size_t)N, sim->S[1], (size_t)N);
    sim->snap_t[slot] = sim->t;
    return 0;
}

uint64_t eao_snapshot_time(const eao_sim *sim, int slot)
{
    if (slot < 0 || slot >= sim->n_slots) return 0;
    return sim->snap_t[slot];
}

/* Observables straight from their definitions, eqs. (1), (2), (3) and (7),
 * without the 1/N normalisation. */
void eao_c4_shells(const eao_sim *sim, int n_shells, int64_t *out)
{
    int L = sim->L;
    int64_t N = sim->N;
    for (int k = 0; k < n_shells; ++k) out[k] = 0;
    int8_t *q = (int8_t *)malloc((size_t)N);
    if (!q) return;
    for (int64_t s = 0; s < N; ++s) q[s] = (int8_t)(sim->S[0][s] * sim->S[1][s]);
    for (int rz = 0; rz < L; ++rz) {
        int mz = rz < L - rz ? rz : L - rz;
        for (int ry = 0; ry < L; ++ry) {
            int my = ry < L - ry ? ry : L - ry;
            for (int rx = 0; rx < L; ++rx) {
                int mx = rx < L - rx ? rx : L - rx;
                int k = mx * mx + my * my + mz * mz;
                if (k >= n_shells) continue;
                int64_t acc = 0;
                for (int64_t s = 0; s < N; ++s) {
                    int x, y, z;
                    coords_of(L, s, &x, &y, &z);
                    acc += q[s] * q[site_of(L, x + rx, y + ry, z + rz)];
                }
                out[k] += acc;
            }
        }
    }
    free(q);
}

void eao_measure(const eao_sim *sim, eao_obs *out)
{
    int L = sim->L;
    int64_t N = sim->N;
    out->t = sim->t;
    for (int r = 0; r < 2; ++r) {
        const int8_t *S = sim->S[r];
        int64_t unsat = 0, mag = 0;
        for (int64_t s = 0; s < N; ++s) {
            int x, y, z;
            coords_of(L, s, &x, &y, &z);
            int64_t nb[3] = {site_of(L, x + 1, y, z), site_of(L, x, y + 1, z),
                             site_of(L, x, y, z + 1)};
            for (int d = 0; d < 3; ++d)
                if (sim->J[3 * s + d] * S[s] * S[nb[d]] < 0) unsat += 1;
            mag += S[s];
        }
        out->unsat[r] = unsat;
        out->mag[r] = mag;
    }
    int64_t ov = 0;
    for (int64_t s = 0; s < N; ++s) ov += sim->S[0][s] * sim->S[1][s];
    out->overlap = ov;

    if (out->autocorr) {
        for (int r = 0; r < 2; ++r) {
            for (int k = 0; k < sim->n_slots; ++k) {
                const int8_t *ref = sim->snap + ((size_t)k * 2 + (size_t)r) * (size_t)N;
                int64_t a = 0;
                for (int64_t s = 0; s < N; ++s) a += sim->S[r][s] * ref[s];
                out->autocorr[r * sim->n_slots + k] = a;
            }
        }
    }

    if (out->c4) {
        int half = L / 2;
        for (int d = 0; d < 3; ++d) {
            for (int rho = 0; rho <= half; ++rho) {
                int64_t acc = 0;
                for (int64_t s = 0; s < N; ++s) {
                    int x, y, z;
                    coords_of(L, s, &x, &y, &z);
                    int64_t o = site_of(L, x + (d == 0) * rho, y + (d == 1) * rho,
                                        z + (d == 2) * rho);
                    int q_s = sim->S[0][s] * sim->S[1][s];
                    int q_o = sim->S[0][o] * sim->S[1][o];
                    acc += q_s * q_o;
                }
                out->c4[d * (half + 1) + rho] = acc;
            }
        }
    }
}

void eao_get_spins(const eao_sim *sim, int r, int8_t *S)
{
    memcpy(S, sim->S[r & 1], (size_t)sim->N);
}

void eao_set_spins(eao_sim *sim, int r, const int8_t *S)
{
    memcpy(sim->S[r & 1], S, (size_t)sim->N);
}

void eao_get_bonds(const eao_sim *sim, int8_t *J)
{
    memcpy(J, sim->J, (size_t)(3 * sim->N));
}

void eao_set_bonds(eao_sim *sim, const int8_t *J)
{
    memcpy(sim->J, J, (size_t)(3 * sim->N));
}
