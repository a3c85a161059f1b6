/*
 * potts_oracle.c -- serial CPU oracle for the checkerboard Metropolis sweep of
 * the two-dimensional q-state Potts model (Ferrero, De Francesco, Wolovick,
 * Cannas, "q-state Potts model metastability study using optimized GPU-based
 * Monte Carlo algorithms", arXiv:1101.0876).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product library never calls it
 * and shares no code, header or table generator with it.
 *
 * Every function is written from the paper's definitions, in the order the
 * paper states them, with no blocking, fusion or reordering:
 *   - Hamiltonian H = -J sum_<ij> delta(s_i, s_j), J = 1          (Sec. 2.1, Eq. 1)
 *   - order parameter from N_max = max_v N_v                       (Sec. 2.1, Eq. 7)
 *   - one MCS = N single-spin Metropolis trials                   (Sec. 2.2)
 *   - all sites of one checkerboard colour, then the other        (Sec. 3, opening)
 *   - one integer proposal in {0..q-1} plus one acceptance number (Sec. 3.2)
 *   - per-temperature table of acceptance weights                 (Sec. 5, CPU code)
 *   - the spin is always written back                             (Sec. 5)
 *
 * Readings where the paper leaves a choice open (all documented with the
 * library contract):
 *   - spins are stored 0..q-1 (paper's label s is stored as s-1); the ordered
 *     start is all zeros;
 *   - colour c(x,y) = (x+y) & 1; colour 0 is updated first;
 *   - the proposal is uniform over all q values (the current one included),
 *     drawn as k = floor(w * q / 2^32) from a 32-bit word w;
 *   - acceptance compares a 32-bit word against an integer threshold table
 *     thr[d] = min(floor(exp(-beta d) 2^32), 2^32 - 1), d = 1..4, built in FP64;
 *     a move with dE <= 0 is always accepted;
 *   - random numbers come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 *     SC'11, "Parallel random numbers: as easy as 1, 2, 3"), one block per
 *     (4-byte row chunk, sweep, colour): counter = (t_lo, y*(L/4) + x/4, t_hi,
 *     colour), key = (seed_lo, seed_hi); a site at column x takes the word pair
 *     (w[2b], w[2b+1]) with b = (x/2) & 1 as (proposal, acceptance).  The random
 *     start uses counter (0, y*(L/4) + x/4, 0, 2) and value floor(w[x&3]*q/2^32).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11), written from its published round
 * definition: two 32x32->64 products, each high half XORed with the other
 * counter word and a key word, and a Weyl increment of the key between rounds. */
static void philox_round(uint32_t x[4], const uint32_t k[2])
{
    const uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x[0];
    const uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x[2];
    const uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    const uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    const uint32_t y0 = hi1 ^ x[1] ^ k[0];
    const uint32_t y1 = lo1;
    const uint32_t y2 = hi0 ^ x[3] ^ k[1];
    const uint32_t y3 = lo0;
    x[0] = y0; x[1] = y1; x[2] = y2; x[3] = y3;
}

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(x, k);
    }
    out[0] = x[0]; out[1] = x[1]; out[2] = x[2]; out[3] = x[3];
}

/* ------------------------------------------------------------------------ */
/* Table of acceptance weights for one temperature (Sec. 5: the CPU code keeps
 * precomputed Boltzmann weights per temperature).  Entry d (1..4) is the
 * Metropolis weight exp(-beta*d) scaled to 32 bits, floored, saturated. */
int oracle_threshold_table(double beta, uint32_t thr[4])
{
    if (!(beta >= 0.0) || isinf(beta)) return ORACLE_EINVAL;
    for (int d = 1; d <= 4; ++d) {
        const double weight = exp(-beta * (double)d);
        double scaled = floor(weight * 4294967296.0);
        if (scaled > 4294967295.0) scaled = 4294967295.0;
        thr[d - 1] = (uint32_t)scaled;
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
static int valid_shape(int L, int q)
{
    return L >= 4 && L % 4 == 0 && q >= 2 && q <= 256;
}

/* Lemire multiply-shift: a 32-bit word mapped onto {0..q-1}. */
static uint32_t word_to_value(uint32_t w, int q)
{
    return (uint32_t)(((uint64_t)w * (uint64_t)(uint32_t)q) >> 32);
}

/* Philox words for the chunk holding column x of row y: counter
 * (c0, chunk index, c2, c3). */
static void chunk_words(int L, int x, int y, uint64_t seed, uint32_t c0, uint32_t c2,
                        uint32_t c3, uint32_t w[4])
{
    const uint32_t ctr[4] = {c0, (uint32_t)((uint64_t)y * (uint64_t)(L / 4) + (uint64_t)(x / 4)),
                             c2, c3};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, w);
}

/* Initial condition (Sec. 3, protocol): ordered = every spin in the first
 * state; random = each spin drawn independently and uniformly. */
int oracle_init(int L, int q, uint64_t seed, int start, uint8_t *spins)
{
    if (!valid_shape(L, q) || spins == NULL || (start != 0 && start != 1)) return ORACLE_EINVAL;
    for (int y = 0; y < L; ++y) {
        for (int x = 0; x < L; ++x) {
            uint8_t value = 0;
            if (start == 1) {
                uint32_t w[4];
                chunk_words(L, x, y, seed, 0u, 0u, 2u, w);
                value = (uint8_t)word_to_value(w[x & 3], q);
            }
            spins[(size_t)y * (size_t)L + (size_t)x] = value;
        }
    }
    return ORACLE_OK;
}

/* One Metropolis trial for a single site (Sec. 3.2 and Eq. 1).  nb holds the
 * four nearest-neighbour spins; returns the spin after the trial.  Exported so
 * that the tests can probe the decision rule directly. */
int oracle_site_update(int q, int s, const uint8_t nb[4], uint32_t w_prop, uint32_t w_acc,
                       const uint32_t thr[4])
{
    const int k = (int)word_to_value(w_prop, q);
    int equal_now = 0, equal_new = 0;
    for (int j = 0; j < 4; ++j) {
        if (nb[j] == s) ++equal_now;
        if (nb[j] == k) ++equal_new;
    }
    /* H = -(satisfied bonds), so the energy change of s -> k is the number of
     * satisfied bonds lost: equal_now - equal_new. */
    const int dE = equal_now - equal_new;
    int accept;
    if (dE <= 0) accept = 1;
    else accept = (w_acc < thr[dE - 1]);
    return accept ? k : s;
}

/* Update every site of one colour, in the given visiting order (NULL = row
 * major).  Sites of one colour only have neighbours of the other colour, so the
 * order cannot change the result; the tests check exactly that. */
int oracle_half_sweep(int L, int q, uint64_t seed, uint64_t t, int colour, const uint32_t thr[4],
                      uint8_t *spins, const int64_t *order)
{
    if (!valid_shape(L, q) || spins == NULL || thr == NULL || (colour != 0 && colour != 1))
        return ORACLE_EINVAL;
    const int64_t n = (int64_t)L * (int64_t)L;
    for (int64_t visit = 0; visit < n; ++visit) {
        const int64_t i = order ? order[visit] : visit;
        if (i < 0 || i >= n) return ORACLE_EINVAL;
        const int x = (int)(i % L), y = (int)(i / L);
        if (((x + y) & 1) != colour) continue;
        const uint8_t nb[4] = {
            spins[(size_t)y * L + (size_t)((x + 1) % L)],          /* right */
            spins[(size_t)y * L + (size_t)((x + L - 1) % L)],      /* left  */
            spins[(size_t)((y + 1) % L) * L + (size_t)x],          /* down  */
            spins[(size_t)((y + L - 1) % L) * L + (size_t)x],      /* up    */
        };
        uint32_t w[4];
        chunk_words(L, x, y, seed, (uint32_t)t, (uint32_t)(t >> 32), (uint32_t)colour, w);
        const int b = (x / 2) & 1;
        const int s = spins[(size_t)y * L + (size_t)x];
        spins[(size_t)y * L + (size_t)x] =
            (uint8_t)oracle_site_update(q, s, nb, w[2 * b], w[2 * b + 1], thr);
    }
    return ORACLE_OK;
}

/* Energy and order-parameter inputs by direct definition (Eq. 1, Eq. 7):
 * e_sat = number of satisfied nearest-neighbour bonds (H = -e_sat), each bond
 * counted once through the right and down neighbours; hist[v] = N_v. */
int oracle_observables(int L, int q, const uint8_t *spins, int64_t *e_sat, int64_t *hist)
{
    if (!valid_shape(L, q) || spins == NULL) return ORACLE_EINVAL;
    int64_t bonds = 0;
    if (hist) memset(hist, 0, sizeof(int64_t) * (size_t)q);
    for (int y = 0; y < L; ++y) {
        for (int x = 0; x < L; ++x) {
            const uint8_t s = spins[(size_t)y * L + x];
            if (s == spins[(size_t)y * L + (size_t)((x + 1) % L)]) ++bonds;
            if (s == spins[(size_t)((y + 1) % L) * L + x]) ++bonds;
            if (hist) {
                if (s >= q) return ORACLE_EINVAL;
                ++hist[s];
            }
        }
    }
    if (e_sat) *e_sat = bonds;
    return ORACLE_OK;
}

/* n full sweeps (1 MCS each: colour 0 then colour 1), starting at sweep index
 * t0.  If records is not NULL, after sweep j it receives {e_sat, hist[0..q)}
 * at records[j*(1+q)]. */
int oracle_sweeps(int L, int q, uint64_t seed, uint64_t t0, int64_t nsweeps, const uint32_t thr[4],
                  uint8_t *spins, int64_t *records)
{
    if (!valid_shape(L, q) || spins == NULL || thr == NULL || nsweeps < 0) return ORACLE_EINVAL;
    for (int64_t j = 0; j < nsweeps; ++j) {
        const uint64_t t = t0 + (uint64_t)j;
        int rc = oracle_half_sweep(L, q, seed, t, 0, thr, spins, NULL);
        if (rc) return rc;
        rc = oracle_half_sweep(L, q, seed, t, 1, thr, spins, NULL);
        if (rc) return rc;
        if (records) {
            int64_t *rec = records + (size_t)j * (size_t)(1 + q);
            rc = oracle_observables(L, q, spins, &rec[0], &rec[1]);
            if (rc) return rc;
        }
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Heat-bath update (Sec. 7 names other single-spin-flip algorithms as the
 * natural extension of the Metropolis update).  The new value k of a site is
 * drawn with probability proportional to exp(beta n(k)), n(v) = number of the
 * four neighbours equal to v (Eq. 1), whatever the current value.  The
 * contract (readings of this implementation):
 *   - weights are taken relative to the best neighbour count n_max: value v
 *     weighs D[n_max - n(v)], D[0] = 2^32, D[d] = thr[d-1] for d = 1..4 (the
 *     Metropolis table); the common factor exp(beta n_max) cancels and the
 *     total weight Z is at least 2^32;
 *   - values are ranked: the distinct neighbour values in order of first
 *     appearance among (up, down, left, right), then every other value in
 *     increasing order; r = floor(w Z / 2^32) for the site's 32-bit word w,
 *     and k is the first value in the ranking whose cumulative weight exceeds
 *     r;
 *   - w is the word the Metropolis update uses as its proposal, from a block
 *     whose counter word 3 is colour + 4 (a stream of its own). */
int oracle_heatbath_site(int q, const uint8_t nb[4], uint32_t w, const uint32_t thr[4])
{
    int count[256] = {0};
    int seen[256] = {0};
    int rank[256];
    int m = 0, n_max = 0;
    for (int j = 0; j < 4; ++j) ++count[nb[j]];
    for (int v = 0; v < q; ++v)
        if (count[v] > n_max) n_max = count[v];
    for (int j = 0; j < 4; ++j) {
        if (!seen[nb[j]]) {
            seen[nb[j]] = 1;
            rank[m++] = nb[j];
        }
    }
    for (int v = 0; v < q; ++v)
        if (!seen[v]) rank[m++] = v;
    const uint64_t D[5] = {(uint64_t)1 << 32, thr[0], thr[1], thr[2], thr[3]};
    uint64_t Z = 0;
    for (int i = 0; i < q; ++i) Z += D[n_max - count[rank[i]]];
    const uint64_t r = (uint64_t)(((unsigned __int128)w * Z) >> 32);
    uint64_t cum = 0;
    for (int i = 0; i < q; ++i) {
        cum += D[n_max - count[rank[i]]];
        if (r < cum) return rank[i];
    }
    return rank[q - 1]; /* not reached: r < Z */
}

/* One colour of a heat-bath sweep; sites of one colour only have neighbours
 * of the other colour (Sec. 3), so they are visited in row-major order. */
int oracle_heatbath_half_sweep(int L, int q, uint64_t seed, uint64_t t, int colour, const uint32_t thr[4],
                               uint8_t *spins)
{
    if (!valid_shape(L, q) || spins == NULL || thr == NULL || (colour != 0 && colour != 1))
        return ORACLE_EINVAL;
    for (int y = 0; y < L; ++y) {
        for (int x = 0; x < L; ++x) {
            if (((x + y) & 1) != colour) continue;
            const uint8_t nb[4] = {
                spins[(size_t)((y + L - 1) % L) * L + (size_t)x],      /* up    */
                spins[(size_t)((y + 1) % L) * L + (size_t)x],          /* down  */
                spins[(size_t)y * L + (size_t)((x + L - 1) % L)],      /* left  */
                spins[(size_t)y * L + (size_t)((x + 1) % L)],          /* right */
            };
            uint32_t w[4];
            chunk_words(L, x, y, seed, (uint32_t)t, (uint32_t)(t >> 32), (uint32_t)colour + 4u, w);
            const int b = (x / 2) & 1;
            spins[(size_t)y * L + (size_t)x] = (uint8_t)oracle_heatbath_site(q, nb, w[2 * b], thr);
        }
    }
    return ORACLE_OK;
}

/* n heat-bath sweeps from sweep index t0, records as oracle_sweeps. */
int oracle_heatbath_sweeps(int L, int q, uint64_t seed, uint64_t t0, int64_t nsweeps, const uint32_t thr[4],
                           uint8_t *spins, int64_t *records)
{
    if (!valid_shape(L, q) || spins == NULL || thr == NULL || nsweeps < 0) return ORACLE_EINVAL;
    for (int64_t j = 0; j < nsweeps; ++j) {
        const uint64_t t = t0 + (uint64_t)j;
        int rc = oracle_heatbath_half_sweep(L, q, seed, t, 0, thr, spins);
        if (rc) return rc;
        rc = oracle_heatbath_half_sweep(L, q, seed, t, 1, thr, spins);
        if (rc) return rc;
        if (records) {
            int64_t *rec = records + (size_t)j * (size_t)(1 + q);
            rc = oracle_observables(L, q, spins, &rec[0], &rec[1]);
            if (rc) return rc;
        }
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* The same chain restricted to an h-by-w window of an L-by-L lattice whose
 * top-left corner is (x0, y0) (coordinates wrap periodically).  The window
 * starts from the initial condition and runs nsweeps sweeps from t = 0 with
 * the random words of the full lattice.  Sites outside the window are unknown,
 * so each half sweep spoils one more ring of the window; after nsweeps sweeps
 * only sites at least 2*nsweeps from the window edge equal the full-lattice
 * chain.  The caller reads those only.  This lets the tests check samples of
 * very large lattices one window at a time. */
int oracle_window(int L, int q, uint64_t seed, int start, int64_t nsweeps, const uint32_t thr[4],
                  int x0, int y0, int h, int w, uint8_t *out)
{
    if (!valid_shape(L, q) || out == NULL || thr == NULL || h < 1 || w < 1 || h > L || w > L ||
        x0 < 0 || y0 < 0 || x0 >= L || y0 >= L || nsweeps < 0 || (start != 0 && start != 1))
        return ORACLE_EINVAL;
    uint8_t *cur = (uint8_t *)malloc((size_t)h * (size_t)w);
    if (!cur) return ORACLE_ENOMEM;
    for (int r = 0; r < h; ++r) {
        for (int c = 0; c < w; ++c) {
            const int x = (x0 + c) % L, y = (y0 + r) % L;
            uint8_t value = 0;
            if (start == 1) {
                uint32_t wd[4];
                chunk_words(L, x, y, seed, 0u, 0u, 2u, wd);
                value = (uint8_t)word_to_value(wd[x & 3], q);
            }
            cur[(size_t)r * w + c] = value;
        }
    }
    for (int64_t j = 0; j < nsweeps; ++j) {
        const uint64_t t = (uint64_t)j;
        for (int colour = 0; colour < 2; ++colour) {
            for (int r = 0; r < h; ++r) {
                for (int c = 0; c < w; ++c) {
                    const int x = (x0 + c) % L, y = (y0 + r) % L;
                    if (((x + y) & 1) != colour) continue;
                    /* neighbours outside the window read as the site itself:
                     * any value works, the ring is discarded anyway */
                    const uint8_t self = cur[(size_t)r * w + c];
                    const uint8_t nb[4] = {
                        c + 1 < w ? cur[(size_t)r * w + c + 1] : self,
                        c - 1 >= 0 ? cur[(size_t)r * w + c - 1] : self,
                        r + 1 < h ? cur[(size_t)(r + 1) * w + c] : self,
                        r - 1 >= 0 ? cur[(size_t)(r - 1) * w + c] : self,
                    };
                    uint32_t wd[4];
                    chunk_words(L, x, y, seed, (uint32_t)t, (uint32_t)(t >> 32), (uint32_t)colour, wd);
                    const int b = (x / 2) & 1;
                    cur[(size_t)r * w + c] =
                        (uint8_t)oracle_site_update(q, self, nb, wd[2 * b], wd[2 * b + 1], thr);
                }
            }
        }
    }
    memcpy(out, cur, (size_t)h * (size_t)w);
    free(cur);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Simple-cubic lattice (Sec. 7: the checkerboard update carries over to three
 * dimensions with its two independent sub-lattices).  Contract of this
 * implementation, the 2D one lifted to L x L x L:
 *   - site (x, y, z) at byte (z L + y) L + x, periodic, L >= 4, L % 4 == 0;
 *   - colour (x + y + z) & 1, colour 0 first;
 *   - six neighbours, dE = n(s) - n(k) in -6..6, thresholds for d = 1..6;
 *   - Philox block per (4-byte row chunk, sweep, colour): counter
 *     (t_lo, ((z L + y) L + x) / 4, t_hi, colour + 8); site x takes
 *     (w[2b], w[2b+1]), b = (x/2) & 1; random start: counter
 *     (0, chunk, 0, 10) and value floor(w[x&3] q / 2^32). */
int oracle_threshold_table6(double beta, uint32_t thr[6])
{
    if (!(beta >= 0.0) || isinf(beta)) return ORACLE_EINVAL;
    for (int d = 1; d <= 6; ++d) {
        double scaled = floor(exp(-beta * (double)d) * 4294967296.0);
        if (scaled > 4294967295.0) scaled = 4294967295.0;
        thr[d - 1] = (uint32_t)scaled;
    }
    return ORACLE_OK;
}

static int valid_cube(int L, int q)
{
    return L >= 4 && L % 4 == 0 && (uint64_t)L * L * L / 4 < ((uint64_t)1 << 32) && q >= 2 && q <= 256;
}

static void cube_words(int L, int x, int y, int z, uint64_t seed, uint32_t c0, uint32_t c2, uint32_t c3,
                       uint32_t w[4])
{
    const uint64_t site = ((uint64_t)z * L + (uint64_t)y) * L + (uint64_t)x;
    const uint32_t ctr[4] = {c0, (uint32_t)(site / 4), c2, c3};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, w);
}

static size_t cube_at(int L, int x, int y, int z)
{
    return ((size_t)z * (size_t)L + (size_t)y) * (size_t)L + (size_t)x;
}

int oracle3d_init(int L, int q, uint64_t seed, int start, uint8_t *spins)
{
    if (!valid_cube(L, q) || spins == NULL || (start != 0 && start != 1)) return ORACLE_EINVAL;
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                uint8_t value = 0;
                if (start == 1) {
                    uint32_t w[4];
                    cube_words(L, x, y, z, seed, 0u, 0u, 10u, w);
                    value = (uint8_t)word_to_value(w[x & 3], q);
                }
                spins[cube_at(L, x, y, z)] = value;
            }
    return ORACLE_OK;
}

/* One Metropolis trial with six neighbours (Eq. 1 on the cubic lattice). */
int oracle3d_site_update(int q, int s, const uint8_t nb[6], uint32_t w_prop, uint32_t w_acc,
                         const uint32_t thr[6])
{
    const int k = (int)word_to_value(w_prop, q);
    int equal_now = 0, equal_new = 0;
    for (int j = 0; j < 6; ++j) {
        if (nb[j] == s) ++equal_now;
        if (nb[j] == k) ++equal_new;
    }
    const int dE = equal_now - equal_new;
    const int accept = dE <= 0 ? 1 : (w_acc < thr[dE - 1]);
    return accept ? k : s;
}

int oracle3d_half_sweep(int L, int q, uint64_t seed, uint64_t t, int colour, const uint32_t thr[6],
                        uint8_t *spins)
{
    if (!valid_cube(L, q) || spins == NULL || thr == NULL || (colour != 0 && colour != 1))
        return ORACLE_EINVAL;
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                if (((x + y + z) & 1) != colour) continue;
                const uint8_t nb[6] = {
                    spins[cube_at(L, (x + 1) % L, y, z)], spins[cube_at(L, (x + L - 1) % L, y, z)],
                    spins[cube_at(L, x, (y + 1) % L, z)], spins[cube_at(L, x, (y + L - 1) % L, z)],
                    spins[cube_at(L, x, y, (z + 1) % L)], spins[cube_at(L, x, y, (z + L - 1) % L)],
                };
                uint32_t w[4];
                cube_words(L, x, y, z, seed, (uint32_t)t, (uint32_t)(t >> 32), (uint32_t)colour + 8u, w);
                const int b = (x / 2) & 1;
                const size_t i = cube_at(L, x, y, z);
                spins[i] = (uint8_t)oracle3d_site_update(q, spins[i], nb, w[2 * b], w[2 * b + 1], thr);
            }
    return ORACLE_OK;
}

/* e_sat over the 3N bonds (each counted once through +x, +y, +z) and N_v. */
int oracle3d_observables(int L, int q, const uint8_t *spins, int64_t *e_sat, int64_t *hist)
{
    if (!valid_cube(L, q) || spins == NULL) return ORACLE_EINVAL;
    int64_t bonds = 0;
    if (hist) memset(hist, 0, sizeof(int64_t) * (size_t)q);
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                const uint8_t s = spins[cube_at(L, x, y, z)];
                bonds += s == spins[cube_at(L, (x + 1) % L, y, z)];
                bonds += s == spins[cube_at(L, x, (y + 1) % L, z)];
                bonds += s == spins[cube_at(L, x, y, (z + 1) % L)];
                if (hist) {
                    if (s >= q) return ORACLE_EINVAL;
                    ++hist[s];
                }
            }
    if (e_sat) *e_sat = bonds;
    return ORACLE_OK;
}

int oracle3d_sweeps(int L, int q, uint64_t seed, uint64_t t0, int64_t nsweeps, const uint32_t thr[6],
                    uint8_t *spins, int64_t *records)
{
    if (!valid_cube(L, q) || spins == NULL || thr == NULL || nsweeps < 0) return ORACLE_EINVAL;
    for (int64_t j = 0; j < nsweeps; ++j) {
        const uint64_t t = t0 + (uint64_t)j;
        int rc = oracle3d_half_sweep(L, q, seed, t, 0, thr, spins);
        if (rc) return rc;
        rc = oracle3d_half_sweep(L, q, seed, t, 1, thr, spins);
        if (rc) return rc;
        if (records) {
            int64_t *rec = records + (size_t)j * (size_t)(1 + q);
            rc = oracle3d_observables(L, q, spins, &rec[0], &rec[1]);
            if (rc) return rc;
        }
    }
    return ORACLE_OK;
}

/* The cubic chain restricted to a d x d x d window with corner (x0, y0, z0)
 * (coordinates wrap), from the initial condition at t = 0, with the random
 * words of the full lattice (the 2D window above, one dimension up): after
 * nsweeps sweeps only sites at least 2*nsweeps from every face of the window
 * equal the full-lattice chain. */
int oracle3d_window(int L, int q, uint64_t seed, int start, int64_t nsweeps, const uint32_t thr[6], int x0,
                    int y0, int z0, int d, uint8_t *out)
{
    if (!valid_cube(L, q) || out == NULL || thr == NULL || d < 1 || d > L || x0 < 0 || y0 < 0 || z0 < 0 ||
        x0 >= L || y0 >= L || z0 >= L || nsweeps < 0 || (start != 0 && start != 1))
        return ORACLE_EINVAL;
    for (int k = 0; k < d; ++k)
        for (int j = 0; j < d; ++j)
            for (int i = 0; i < d; ++i) {
                const int x = (x0 + i) % L, y = (y0 + j) % L, z = (z0 + k) % L;
                uint8_t value = 0;
                if (start == 1) {
                    uint32_t w[4];
                    cube_words(L, x, y, z, seed, 0u, 0u, 10u, w);
                    value = (uint8_t)word_to_value(w[x & 3], q);
                }
                out[cube_at(d, i, j, k)] = value;
            }
    for (int64_t n = 0; n < nsweeps; ++n) {
        const uint64_t t = (uint64_t)n;
        for (int colour = 0; colour < 2; ++colour)
            for (int k = 0; k < d; ++k)
                for (int j = 0; j < d; ++j)
                    for (int i = 0; i < d; ++i) {
                        const int x = (x0 + i) % L, y = (y0 + j) % L, z = (z0 + k) % L;
                        if (((x + y + z) & 1) != colour) continue;
                        /* neighbours outside the window read as the site itself
                         * (those faces are discarded) */
                        const uint8_t self = out[cube_at(d, i, j, k)];
                        const uint8_t nb[6] = {
                            i + 1 < d ? out[cube_at(d, i + 1, j, k)] : self,
                            i > 0 ? out[cube_at(d, i - 1, j, k)] : self,
                            j + 1 < d ? out[cube_at(d, i, j + 1, k)] : self,
                            j > 0 ? out[cube_at(d, i, j - 1, k)] : self,
                            k + 1 < d ? out[cube_at(d, i, j, k + 1)] : self,
                            k > 0 ? out[cube_at(d, i, j, k - 1)] : self,
                        };
                        uint32_t w[4];
                        cube_words(L, x, y, z, seed, (uint32_t)t, (uint32_t)(t >> 32), (uint32_t)colour + 8u, w);
                        const int b = (x / 2) & 1;
                        out[cube_at(d, i, j, k)] =
                            (uint8_t)oracle3d_site_update(q, self, nb, w[2 * b], w[2 * b + 1], thr);
                    }
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* First and second neighbours on the square lattice (Sec. 7: with
 * second-neighbour couplings the lattice splits into nine independent
 * sub-lattices instead of two).  Contract of this implementation:
 *   - H = -sum_<ij> delta(s_i, s_j) - j2 sum_<<ij>> delta(s_i, s_j): the four
 *     nearest neighbours with coupling 1 and the four diagonal neighbours
 *     with coupling j2 (Eq. 1 extended to second neighbours);
 *   - L x L periodic, L % 12 == 0 (three colours per axis, 4-byte chunks);
 *   - colour c = 3 (y mod 3) + (x mod 3); one sweep updates colours 0..8 in
 *     turn (two sites of one colour are at least three apart along an axis,
 *     so neither is a first or second neighbour of the other);
 *   - dE = (n1(s) - n1(k)) + j2 (n2(s) - n2(k)) with n1/n2 the numbers of
 *     nearest/diagonal neighbours equal to a value; the table holds, for
 *     d1 = n1(s) - n1(k) and d2 = n2(s) - n2(k) in -4..4, entry
 *     (d1 + 4) * 9 + (d2 + 4) = 2^32 when dE <= 0 (always accept), else
 *     min(floor(exp(-beta dE) 2^32), 2^32 - 1); a move is accepted iff
 *     w_acc < entry;
 *   - Philox block per (6-byte row segment, sweep, colour): counter
 *     (t_lo, y L/6 + x/6, t_hi, 16 + colour); site x takes (w[2b], w[2b+1]),
 *     b = (x/3) & 1 (a segment holds exactly two sites of each colour, at
 *     x mod 6 = x mod 3 and x mod 3 + 3);
 *   - the initial conditions are those of the nearest-neighbour lattice;
 *   - records {e1, e2, hist[q]}: satisfied nearest-neighbour bonds (2N),
 *     satisfied diagonal bonds (2N) and the populations. */
static void segment_words(int L, int x, int y, uint64_t seed, uint32_t c0, uint32_t c2, uint32_t c3, uint32_t w[4])
{
    const uint32_t ctr[4] = {c0, (uint32_t)((uint64_t)y * (uint64_t)(L / 6) + (uint64_t)(x / 6)), c2, c3};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, w);
}

static int valid_nnn(int L, int q)
{
    return L >= 12 && L % 12 == 0 && (uint64_t)L * (uint64_t)L / 4 < ((uint64_t)1 << 32) && q >= 2 && q <= 256;
}

int oracle_nnn_table(double beta, double j2, uint64_t thr[81])
{
    if (!(beta >= 0.0) || isinf(beta) || !isfinite(j2) || thr == NULL) return ORACLE_EINVAL;
    for (int d1 = -4; d1 <= 4; ++d1)
        for (int d2 = -4; d2 <= 4; ++d2) {
            const double de = (double)d1 + j2 * (double)d2;
            uint64_t entry;
            if (de <= 0.0) {
                entry = (uint64_t)1 << 32;
            } else {
                double scaled = floor(exp(-beta * de) * 4294967296.0);
                if (scaled > 4294967295.0) scaled = 4294967295.0;
                entry = (uint64_t)scaled;
            }
            thr[(d1 + 4) * 9 + (d2 + 4)] = entry;
        }
    return ORACLE_OK;
}

/* One Metropolis trial: nb1 the four nearest, nb2 the four diagonal neighbours. */
int oracle_nnn_site_update(int q, int s, const uint8_t nb1[4], const uint8_t nb2[4], uint32_t w_prop,
                           uint32_t w_acc, const uint64_t thr[81])
{
    const int k = (int)word_to_value(w_prop, q);
    int n1s = 0, n1k = 0, n2s = 0, n2k = 0;
    for (int j = 0; j < 4; ++j) {
        n1s += nb1[j] == s;
        n1k += nb1[j] == k;
        n2s += nb2[j] == s;
        n2k += nb2[j] == k;
    }
    const int d1 = n1s - n1k, d2 = n2s - n2k;
    return (uint64_t)w_acc < thr[(d1 + 4) * 9 + (d2 + 4)] ? k : s;
}

int oracle_nnn_colour_pass(int L, int q, uint64_t seed, uint64_t t, int colour, const uint64_t thr[81],
                           uint8_t *spins)
{
    if (!valid_nnn(L, q) || spins == NULL || thr == NULL || colour < 0 || colour > 8) return ORACLE_EINVAL;
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x) {
            if (3 * (y % 3) + (x % 3) != colour) continue;
            const int xl = (x + L - 1) % L, xr = (x + 1) % L, yu = (y + L - 1) % L, yd = (y + 1) % L;
            const uint8_t nb1[4] = {spins[(size_t)y * L + xr], spins[(size_t)y * L + xl], spins[(size_t)yd * L + x],
                                    spins[(size_t)yu * L + x]};
            const uint8_t nb2[4] = {spins[(size_t)yu * L + xl], spins[(size_t)yu * L + xr],
                                    spins[(size_t)yd * L + xl], spins[(size_t)yd * L + xr]};
            uint32_t w[4];
            segment_words(L, x, y, seed, (uint32_t)t, (uint32_t)(t >> 32), 16u + (uint32_t)colour, w);
            const int b = (x / 3) & 1;
            const size_t i = (size_t)y * L + x;
            spins[i] = (uint8_t)oracle_nnn_site_update(q, spins[i], nb1, nb2, w[2 * b], w[2 * b + 1], thr);
        }
    return ORACLE_OK;
}

/* e1 over the 2N nearest-neighbour bonds (right, down), e2 over the 2N
 * diagonal bonds (down-right, down-left), and N_v. */
int oracle_nnn_observables(int L, int q, const uint8_t *spins, int64_t *e1, int64_t *e2, int64_t *hist)
{
    if (!valid_nnn(L, q) || spins == NULL) return ORACLE_EINVAL;
    int64_t b1 = 0, b2 = 0;
    if (hist) memset(hist, 0, sizeof(int64_t) * (size_t)q);
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x) {
            const uint8_t s = spins[(size_t)y * L + x];
            const int xr = (x + 1) % L, xl = (x + L - 1) % L, yd = (y + 1) % L;
            b1 += s == spins[(size_t)y * L + xr];
            b1 += s == spins[(size_t)yd * L + x];
            b2 += s == spins[(size_t)yd * L + xr];
            b2 += s == spins[(size_t)yd * L + xl];
            if (hist) {
                if (s >= q) return ORACLE_EINVAL;
                ++hist[s];
            }
        }
    if (e1) *e1 = b1;
    if (e2) *e2 = b2;
    return ORACLE_OK;
}

int oracle_nnn_sweeps(int L, int q, uint64_t seed, uint64_t t0, int64_t nsweeps, const uint64_t thr[81],
                      uint8_t *spins, int64_t *records)
{
    if (!valid_nnn(L, q) || spins == NULL || thr == NULL || nsweeps < 0) return ORACLE_EINVAL;
    for (int64_t j = 0; j < nsweeps; ++j) {
        const uint64_t t = t0 + (uint64_t)j;
        for (int colour = 0; colour < 9; ++colour) {
            const int rc = oracle_nnn_colour_pass(L, q, seed, t, colour, thr, spins);
            if (rc) return rc;
        }
        if (records) {
            int64_t *rec = records + (size_t)j * (size_t)(2 + q);
            const int rc = oracle_nnn_observables(L, q, spins, &rec[0], &rec[1], &rec[2]);
            if (rc) return rc;
        }
    }
    return ORACLE_OK;
}
