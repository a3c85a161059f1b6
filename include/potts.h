/*
 * potts.h -- C ABI of the MI355X (gfx950) library for checkerboard Metropolis
 * Monte Carlo of the two-dimensional ferromagnetic q-state Potts model
 * (Ferrero, De Francesco, Wolovick, Cannas, arXiv:1101.0876).
 *
 * Model (Sec. 2.1, Eq. 1): H = -sum over nearest-neighbour bonds of
 * delta(s_i, s_j) on an L x L periodic square lattice, J = k_B = 1.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Lattice: L x L uint8 spins, row-major, site (x, y) at byte y*L + x,
 *    values 0..q-1 (the paper's label s is stored as s-1).  4 <= L, L % 4 == 0,
 *    2 <= q <= 256 (one byte per spin, Sec. 3.3).
 *  - One sweep (one MCS, N = L*L trials, Sec. 2.2) updates every site with
 *    (x+y) even, then every site with (x+y) odd (checkerboard, Sec. 3).
 *  - Random numbers: Philox4x32-10 (Salmon et al., SC'11), key = seed, one
 *    block per (4-byte row chunk, sweep, colour): counter = (t_lo,
 *    y*(L/4) + x/4, t_hi, colour).  Site x uses words (w[2b], w[2b+1]), b = (x/2) & 1,
 *    as (proposal, acceptance).  The proposal is k = floor(w*q / 2^32), uniform
 *    over all q values (Sec. 3.2: one integer in 0..q-1 and one acceptance
 *    number).  Random start: counter (0, y*(L/4) + x/4, 0, 2), spin =
 *    floor(w[x&3]*q / 2^32).  t counts the sweeps this state has done.
 *    Results are therefore a pure function of (L, q, seed, start, beta
 *    schedule) and do not depend on how kernels are launched.
 *  - Acceptance: dE = n(s) - n(k), n(v) = number of the 4 neighbours equal to
 *    v; a move is accepted if dE <= 0 or w_acc < thr[dE-1], where
 *    thr[d-1] = min(floor(exp(-beta d) 2^32), 2^32 - 1) (per-temperature
 *    Boltzmann table, Sec. 5).  The spin is always written (Sec. 5).
 *  - Records: after every sweep the library stores {e_sat, hist[0..q)} as
 *    int64, where e_sat = number of satisfied bonds (H = -e_sat) and hist[v]
 *    = N_v, the input of the order parameter (Eq. 7).  They are reduced inside
 *    the sweep kernels (Sec. 3.4 does it in separate kernels; Sec. 7 suggests
 *    on-the-fly accumulation).
 *
 * Return codes: 0 on success, a negative POTTS_E* code otherwise.  The library
 * never aborts; the text of the last error of the calling thread is available
 * from potts_last_error().  Every HIP call is checked (Sec. 3.5).
 *
 * Threading: a state is not thread-safe; distinct states may be used from
 * distinct threads and run concurrently on distinct streams.
 */
#ifndef POTTS_H
#define POTTS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define POTTS_OK 0
#define POTTS_EINVAL (-1)  /* bad argument: L, q, beta, nsweeps, NULL pointer */
#define POTTS_ENOMEM (-2)  /* device or host allocation failed                */
#define POTTS_EDEVICE (-3) /* a HIP call failed; see potts_last_error()       */
#define POTTS_ERANGE (-4)  /* index outside the record ring, or too large     */
#define POTTS_EIO (-5)     /* checkpoint file could not be read or written    */

#define POTTS_QMAX 256

typedef struct potts_state potts_state;

typedef enum { POTTS_ORDERED = 0, POTTS_RANDOM = 1 } potts_start;

/* Energy and order-parameter sums of the current configuration. */
typedef struct {
    int64_t t;                 /* sweeps done by the state                  */
    int64_t e_sat;             /* satisfied bonds; H = -e_sat (Eq. 1)       */
    int64_t nmax;              /* max_v hist[v] (Eq. 7)                     */
    int32_t q;
    int32_t L;
    int64_t hist[POTTS_QMAX];  /* hist[v] = N_v, valid for v < q            */
} potts_obs;

/* Derived FP64 observables of a window of n consecutive sweep records
 * (Sec. 2.1, Sec. 4): e = <H>/N, C = beta^2 (<H^2> - <H>^2)/N,
 * V_L = 1 - <H^4>/(3 <H^2>^2) (Eq. 9), m = <(q N_max/N - 1)/(q-1)> (Eq. 7),
 * chi = N beta (<m^2> - <m>^2) (Eq. 11).  The integer moments are summed
 * exactly on the device and each result is rounded once. */
typedef struct {
    int64_t n;
    double e;
    double C;
    double V_L;
    double m;
    double chi;
} potts_summary;

/* Creates a state: allocates the lattice, a second lattice buffer and a ring of
 * per-sweep records (4096 slots; potts_init_ex: records_capacity rounded up to
 * a power of two, 0 selects 4096; at most 2^40) on the current HIP
 * device, creates a stream, and writes the initial condition (Sec. 3:
 * heating starts ordered, cooling starts random).
 * Errors: EINVAL (L < 4, L % 4 != 0, q outside 2..256, bad start, out NULL),
 * ERANGE (L*L/4 >= 2^32), ENOMEM, EDEVICE.  On error *out is NULL. */
int potts_init(int32_t L, int32_t q, uint64_t seed, potts_start start, potts_state **out);

/* As potts_init, on the caller's stream and optionally on caller-owned device
 * buffers.  hip_stream is a hipStream_t (NULL = the default stream); the state
 * never destroys it.
 *   dev_spins, dev_spins2 both non-NULL: caller-owned buffers of at least L*L
 *     bytes each (bytes gives the size of each), which must outlive the state.
 *     dev_spins holds the row-major lattice (byte y*L + x = site (x, y)) from
 *     the end of every call to the start of the next one, in stream order: a
 *     caller may read it, or write values 0..q-1 into it, between calls
 *     (ordered on hip_stream), and the next sweep starts from what it holds.
 *     dev_spins2 is the library's scratch (the colour-split copy a sweep call
 *     works on).  Neither may be touched while a call's work is in flight.
 *   both NULL: the library allocates and owns both buffers (as potts_init),
 *     and keeps the colour-split copy between calls; the row-major lattice is
 *     then read through potts_device_spins or potts_get_spins.
 *   one NULL: EINVAL.
 * The records ring is owned by the library in every case. */
int potts_init_ex(int32_t L, int32_t q, uint64_t seed, potts_start start, void *dev_spins,
                  void *dev_spins2, size_t bytes, void *hip_stream, int64_t records_capacity,
                  potts_state **out);

/* Runs nsweeps Metropolis sweeps at inverse temperature beta, asynchronously on
 * the state's stream; records one {e_sat, hist} per sweep.  The threshold
 * table is rebuilt only when beta changes.
 * Errors: EINVAL (s NULL, beta < 0 or not finite, nsweeps < 0), ERANGE (the
 * sweep counter would overflow), EDEVICE. */
int potts_sweep(potts_state *s, double beta, int64_t nsweeps);

/* As potts_sweep with a caller-supplied threshold table thr[0..3] (d = 1..4). */
int potts_sweep_thr(potts_state *s, const uint32_t thr[4], int64_t nsweeps);

/* Heat-bath sweeps (Sec. 7 names other single-spin-flip algorithms as the
 * extension of the Metropolis update): each site of colour 0, then of colour
 * 1, takes a new value k drawn with probability proportional to
 * exp(beta n(k)), n(k) = number of its 4 neighbours equal to k, whatever its
 * current value.  Contract: value v weighs D[n_max - n(v)] with n_max the
 * largest neighbour count, D[0] = 2^32 and D[d] = thr[d-1] (the table of
 * potts_threshold_table); values are ranked as the distinct neighbour values
 * in order of first appearance among (up, down, left, right), then the other
 * values ascending; with Z the total weight and w the site's word (the word
 * the Metropolis update uses as its proposal, from a block with counter word
 * 3 = colour + 4), k is the first value in the ranking whose cumulative
 * weight exceeds floor(w Z / 2^32).  Records, the sweep counter t and the
 * state are shared with potts_sweep, so both kinds of sweep can be mixed.
 * Asynchronous on the state's stream; any L % 4 == 0.
 * Errors: as potts_sweep. */
int potts_sweep_heatbath(potts_state *s, double beta, int64_t nsweeps);
/* The same with a caller-supplied table. */
int potts_sweep_heatbath_thr(potts_state *s, const uint32_t thr[4], int64_t nsweeps);

/* Launch tuning; results never depend on it (the random numbers are keyed by
 * site and sweep, not by thread).  kernel: 0 = automatic, 1 = the 16-byte strip
 * kernel (needs L % 16 == 0 and L <= 65520, i.e. a lattice below 4 GiB, which its
 * 32-bit buffer offsets address), 2 = the 4-byte chunk kernel (any L; the
 * automatic choice for L = 65536),
 * 3 = the LDS-resident kernel (L % 16 == 0, L <= 256: one workgroup keeps the
 * lattice in LDS and runs all sweeps of a call in one launch), 4 = the
 * colour-split kernel (L % 32 == 0, L <= 65520: a call copies the lattice into
 * two colour planes in the second buffer, sweeps there and copies it back;
 * the automatic choice for such L above 2048 that kernel 7 does not take),
 * 5 = the multi-sweep tile kernel (L % 16 == 0, L <= 65520; the automatic
 * choice for 256 < L <= 2048 that kernel 7 does not take: each
 * launch runs several sweeps, one LDS tile
 * per workgroup whose halo is recomputed, and moves the row-major lattice
 * between the state's two buffers; with library-owned buffers they trade
 * roles, so potts_device_spins may return the other one afterwards; shape
 * from potts_tune_tiles), 6 = the LDS-resident kernel with its random words
 * drawn beforehand (L % 16 == 0, L <= 64: a generator kernel over the whole
 * GPU writes each site's proposal and acceptance word for up to 1024 sweeps
 * into a device buffer of about 20 bytes per site and sweep, allocated on
 * first use and held until potts_free, and the one-workgroup kernel reads
 * them instead of computing them; the automatic choice for such L),
 * 7 = persistent sweeps on LDS bands (L % 32 == 0, L <= 16384, a band shape
 * from potts_tune_band whose grid the GPU holds at once; the automatic choice
 * for 2048 <= L <= 4096 when it can take the lattice): each workgroup keeps
 * a band of whole rows of the colour-split lattice in LDS for up to 64 sweeps
 * per cooperative launch and trades its two edge rows with the neighbouring
 * bands after every half sweep (an exchange buffer of 2 x L x L / rows bytes,
 * held until potts_free); every wait on a neighbour is bounded (0.25 s, or
 * the microseconds in the environment variable POTTS_BAND_WAIT_US, read at
 * each sweep call), and one that expires, possible only if the grid was not
 * resident at once or the bound is set too short, is reported as EDEVICE by
 * the next call that sweeps or reads results;
 * strip_rows: rows per strip work item (0 = automatic, else an even divisor of
 * L); max_groups: persistent grid size in workgroups (0 = automatic).
 * Errors: EINVAL. */
int potts_tune(potts_state *s, int32_t kernel, int32_t strip_rows, int32_t max_groups);

/* Shape of the multi-sweep tile kernel (kernel 5): tiles of tx bytes (a
 * multiple of 16 dividing L) by ty rows (even, dividing L), `sweeps` sweeps
 * per launch (1..8; the tile reads 2 x sweeps halo rows above and below and
 * 16 halo bytes left and right, and one tile with its halo must fit in
 * 44 KiB of LDS); 0 for any of them = automatic (tx: the largest of 256 ..
 * 16 up to L/8 dividing L, ty: 16 rows up to L = 1024 and 32 above, or the
 * largest even divisor below, 4 sweeps).  Results never depend on it.
 * Errors: EINVAL (a shape the lattice cannot take; the old one is kept). */
int potts_tune_tiles(potts_state *s, int32_t tx, int32_t ty, int32_t sweeps);

/* Shape of the band kernel (kernel 7): `rows` rows per band (even, dividing
 * L; L / rows workgroups) of `block` lanes (256, 512 or 1024, at least
 * L / 16); 0 for both = automatic (the first of 8, 16, 4, 32, 2 rows whose
 * grid the GPU holds at once, the fewest lanes that give each item of a half
 * sweep its own, else 1024); block 0 with rows > 0 = that rule for block.  A
 * band with its two halo rows (L x (rows + 2) bytes) must fit in 136 KiB of
 * LDS.  Results never depend on it.  Errors: EINVAL (a shape the lattice or
 * the GPU cannot take; the old one is kept). */
int potts_tune_band(potts_state *s, int32_t rows, int32_t block);

/* Occupancy of the colour-split kernel: 0 = the compiler's register budget
 * (the default), 8 = at most 64 VGPRs so that 8 waves fit on each SIMD (the
 * variant exists for q <= 16; other q keep the default).  Results never
 * depend on it.  Errors: EINVAL (s NULL, waves_per_simd not 0 or 8). */
int potts_tune_occupancy(potts_state *s, int32_t waves_per_simd);

/* Graph replay of colour-split sweeps: with sweeps > 0, a sweep call of at
 * least that many sweeps captures the launches of `sweeps` sweeps once into
 * a hipGraph (kept while the launch shape and table form stay the same) and
 * replays it, the remainder launched directly; 0 (the default) launches every
 * sweep directly.  Needs a stream that can be captured (not the legacy NULL
 * stream).  Results never depend on it.  Errors: EINVAL (sweeps outside
 * 0 .. 4096). */
int potts_tune_graph(potts_state *s, int32_t sweeps);

/* The table potts_sweep uses for beta: thr[d-1] = min(floor(exp(-beta d)
 * 2^32), 2^32-1), computed on the host in FP64.  Errors: EINVAL. */
int potts_threshold_table(double beta, uint32_t thr[4]);

/* One colour half of sweep t (Sec. 3: checkerboard update, Sec. 3.2: one
 * proposal and one acceptance number per site) over a row slab of an L x L
 * lattice: the share of one device when the lattice is split into horizontal
 * slabs.  Because the random words are keyed by global (x, y, t), a lattice
 * swept slab by slab gives the bits of potts_sweep for any slab count.
 *   dev_slab: device, (h+2) x L bytes, row-major.  Row 0 holds global row
 *     (y0-1) mod L, rows 1..h global rows y0 .. y0+h-1, row h+1 global row
 *     (y0+h) mod L.  Rows 1..h are updated in place (sites with (x+y) & 1 ==
 *     colour); rows 0 and h+1 (halos) are only read, and the caller refreshes
 *     them from the neighbouring slabs before every half sweep.
 *   thr: the threshold table of the sweep's beta (potts_threshold_table).
 *   dev_ring: device, ring_slots (a power of two >= 2) slots of 1+q int64.
 *     Both calls of sweep t add this slab's share of the sweep's record into
 *     slot t mod ring_slots: colour 0 the populations of its updated sites,
 *     colour 1 those of its own sites and [0] the satisfied bonds with their
 *     colour-1 end in the slab ([1+v]: sites in state v; summed over the
 *     slabs, the sweep's {e_sat, hist}).  Colour 1 also zeroes slot (t+1) mod
 *     ring_slots for the next sweep.  Slot t must be zero before the colour-0
 *     call of sweep t.
 *   hip_stream: hipStream_t (NULL = default stream); asynchronous.
 * Needs L % 16 == 0, 16 <= L <= 65536, 2 <= q <= 256, h and y0 even,
 * h >= 2, y0 + h <= L, and a slab below 4 GiB ((h+2) L < 2^32).  Errors: EINVAL, EDEVICE. */
int potts_slab_half_sweep(uint8_t *dev_slab, int32_t L, int32_t h, int64_t y0, int32_t q, uint64_t seed,
                          int64_t t, int32_t colour, const uint32_t thr[4], int64_t *dev_ring,
                          int64_t ring_slots, void *hip_stream);

/* The records of a lattice swept slab by slab: record r (r = 0 .. n-1) of
 * sweep t0 + r is the sum over the nslabs slab rings of slot (t0 + r) %
 * ring_slots ({e_sat share, hist share}, 1+q int64 each), written to
 * dev_out[r*(1+q) .. ].  dev_rings: device, the nslabs rings stored one after
 * another (ring g at dev_rings + g * ring_slots * (1+q)), as the slabs' calls
 * of potts_slab_half_sweep filled them.  Asynchronous on hip_stream (a
 * hipStream_t, NULL = the default stream); the caller keeps the records of
 * sweeps t0 .. t0+n-1 in the rings (n <= ring_slots - 1 of them survive a
 * sweep).  Errors: EINVAL (NULL, nslabs < 1, q outside 2..256, ring_slots not
 * a power of two >= 2, t0 < 0, n outside 0..ring_slots), EDEVICE. */
int potts_slab_records(const int64_t *dev_rings, int32_t nslabs, int64_t ring_slots, int32_t q, int64_t t0,
                       int64_t n, int64_t *dev_out, void *hip_stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the sweeps of
 * potts_sweep_thr on the row-major strip kernel, with no state and no
 * allocation.  Bit for bit the sweeps and records potts_sweep_thr gives a
 * state of the same (L, q, seed) whose t is t0 and whose lattice is dev_spins.
 *   dev_spins: device, L*L bytes, row-major, values 0..q-1; sweeps t0 ..
 *     t0+nsweeps-1 update it in place (caller-owned).
 *   thr: host, the threshold table (potts_threshold_table), passed by value
 *     to the kernels.
 *   dev_records: device, nsweeps * (1+q) int64 (caller-owned): record r =
 *     {e_sat, hist[0..q)} of sweep t0 + r.
 *   hip_stream: hipStream_t of the current device (NULL = default stream);
 *     asynchronous, nothing is synchronized.
 * The strip kernel's partial records live in a static device array of
 * 2 x 32 x 272 int64 (139,264 bytes), one per GPU, held until the process
 * ends; every call on a GPU uses it, so calls that overlap on one GPU (on
 * different streams or threads) race and must be ordered by the caller.
 * Each call clears the partial records first.  Calls no hipMalloc, hipFree
 * or allocating library routine and records no memset.
 * Needs L % 16 == 0, 16 <= L <= 65520, 2 <= q <= 256, t0 >= 0.  Errors:
 * EINVAL (NULL, bad shape, negative counts, a stream of another device),
 * ERANGE (t0 + nsweeps overflows, or partial records beyond the static
 * array), EDEVICE. */
int potts_sweep_static(uint8_t *dev_spins, int32_t L, int32_t q, uint64_t seed, int64_t t0,
                       const uint32_t thr[4], int64_t nsweeps, int64_t *dev_records, void *hip_stream);

/* Observables of the current configuration (synchronizes the stream).  Uses
 * the last sweep's record, or measures the lattice if no sweep has run. */
int potts_observables(potts_state *s, potts_obs *out);

/* Measures the current configuration with the standalone observables kernel
 * (independent of the fused reductions; synchronizes). */
int potts_measure(potts_state *s, potts_obs *out);

/* Copies the records of sweeps t0 .. t0+n-1 (sweep t0 = the (t0+1)-th sweep of
 * this state) into out[n*(1+q)] as {e_sat, hist[0..q)} each (synchronizes).
 * Errors: ERANGE if any of them is not (or no longer) in the ring. */
int potts_records(potts_state *s, int64_t t0, int64_t n, int64_t *out);

/* Derived statistics over the records of sweeps t0 .. t0+n-1 at inverse
 * temperature beta (synchronizes).  Errors: ERANGE as potts_records, EINVAL
 * for n < 1. */
int potts_stats(potts_state *s, int64_t t0, int64_t n, double beta, potts_summary *out);

/* Temperature reweighting (Sec. 7 names it; Ferrenberg and Swendsen's
 * single-histogram method): the records of sweeps t0 .. t0+n-1, sampled at
 * inverse temperature beta0, give estimates of the potts_stats observables at
 * each of betas[0..npoints).  Record t gets the weight
 * exp(-(beta - beta0) H_t) = exp((beta - beta0) e_sat_t); out[i] holds the
 * weighted e, C, V_L, m, chi at betas[i] (n = the window length).  FP64 on
 * the device, with the weights and moments taken relative to the window's
 * extreme energy and smallest order parameter (no overflow, no cancellation
 * in the variances); estimates are reliable only where the sampled energy
 * histogram covers the target's.  Synchronizes.
 * Errors: EINVAL (NULL pointer, n < 1, npoints outside 1..65535, a beta < 0
 * or not finite), ERANGE as potts_records, EDEVICE. */
int potts_reweight(potts_state *s, int64_t t0, int64_t n, double beta0, const double *betas, int32_t npoints,
                   potts_summary *out);

/* Grows (or shrinks) the record ring to `capacity` sweeps (2 .. 2^40, rounded
 * up to a power of two).  Records held before the call are discarded.  Synchronizes.  Errors: EINVAL, ENOMEM. */
int potts_reserve_records(potts_state *s, int64_t capacity);

/* Temperature ramp (the simulation protocol of Sec. 3): for k = 0..npoints-1,
 * runs t_equil sweeps and then t_meas sweeps at betas[k], the configuration
 * carrying over from point to point, and writes the derived statistics of the
 * t_meas measurement sweeps to out[k] (caller-owned, npoints entries).
 * Heating starts from the ordered state with beta descending, cooling from the
 * random state with beta ascending; the caller picks the start and order.
 * All work is queued on the state's stream and the call synchronizes once at
 * the end.  The record ring is grown to hold t_meas records when needed.
 * Errors: EINVAL (NULL, npoints < 1, t_equil < 0, t_meas < 1 or > 2^24, bad
 * beta), ENOMEM, EDEVICE. */
int potts_ramp(potts_state *s, const double *betas, int32_t npoints, int64_t t_equil, int64_t t_meas,
               potts_summary *out);

/* Host copies of the lattice (synchronize).  set_spins also sets the sweep
 * counter t; values must be < q (EINVAL otherwise). */
int potts_get_spins(potts_state *s, uint8_t *host_out);
int potts_set_spins(potts_state *s, const uint8_t *host_in, int64_t t);

/* Device pointer of the current lattice, row-major, L*L bytes (valid until the
 * next sweep call).  After colour-split sweeps this first queues the kernel
 * that rebuilds the row-major lattice on the state's stream: read or write the
 * buffer on that stream or after synchronizing it.  The next sweep starts from
 * what the buffer then holds (values must stay below q).  NULL if s is NULL or
 * the kernel could not be queued. */
void *potts_device_spins(potts_state *s);
int64_t potts_time(const potts_state *s);
/* The state's stream (a hipStream_t): the one given to potts_init_ex, or the
 * one potts_init created.  NULL if s is NULL. */
void *potts_stream(const potts_state *s);

/* Checkpoint: (L, q, seed, t, lattice) to a file and back; a resumed state
 * continues with exactly the same random numbers.  Errors: EIO, EINVAL. */
int potts_save(potts_state *s, const char *path);
int potts_load(const char *path, potts_state **out);

/* ---------------------------------------------------------------------------
 * Batches: many independent lattices (replicas, temperatures, sizes) swept
 * together.  Each job gives exactly the spins and records it gives alone
 * (same seed, start, beta, sweeps): the random numbers depend on the site
 * and sweep only.  Jobs with L <= 256 run in the LDS-resident kernel (one
 * workgroup each, all sweeps in one launch); larger jobs share one strip
 * launch per colour and sweep through a workgroup tile table.  The remaining
 * launches of a run are captured in one hipGraph (resident and strip work as
 * two overlapping branches) and replayed.
 */
typedef struct {
    int32_t L, q;        /* L % 16 == 0, 16 <= L <= 65520; 2 <= q <= 256       */
    uint64_t seed;
    int32_t start;       /* potts_start                                        */
    int32_t _pad;
    double beta;         /* one inverse temperature per job                    */
    int64_t nsweeps;     /* sweeps per run, 0 .. 2^31                          */
} potts_job;

typedef struct {
    int64_t t;           /* sweeps done                                        */
    int64_t e_sat;       /* after the last sweep                               */
    int64_t nmax;
    potts_summary stats; /* over the last `window` sweeps (all when window 0)  */
} potts_job_result;

typedef struct {
    int32_t graph;       /* 1: capture the run in a hipGraph and launch it      */
    int32_t tune;        /* 1: time launch shapes on the first sweeps, keep the best */
    int32_t window;      /* summary window in sweeps, 0 = every sweep of the job */
    int32_t strip_rows;  /* fixed strip height (even divisor of L), 0 = automatic */
    void *hip_stream;    /* hipStream_t, NULL = the batch's own stream          */
    const char *tune_cache; /* NULL, or a JSON file of launch shapes (read at
                               create, used with or without `tune`, updated by
                               the tuner; entries measured on other kernel
                               sources are ignored) */
} potts_batch_opts;

typedef struct potts_batch potts_batch;

/* Allocates one arena for all lattices and record rings (every sweep of a run
 * is kept), writes the initial conditions and synchronizes.  opts may be NULL
 * (no graph, no tuning, window 0).  Errors: EINVAL (bad job fields; the message
 * names the job), ENOMEM, EDEVICE. */
int potts_batch_create(const potts_job *jobs, int32_t n, const potts_batch_opts *opts, potts_batch **out);

/* Runs every job for its nsweeps sweeps and waits for the end.  Calling it
 * again continues every job for nsweeps more. Errors: EINVAL, EDEVICE. */
int potts_batch_run(potts_batch *b);

/* Per-job results (caller-owned array of n).  Synchronizes. */
int potts_batch_results(potts_batch *b, potts_job_result *out);

/* Records of sweeps t0 .. t0+n-1 of one job ({e_sat, hist[q]} each) and its
 * lattice (L*L bytes).  Synchronize.  Errors: EINVAL, ERANGE. */
int potts_batch_records(potts_batch *b, int32_t job, int64_t t0, int64_t n, int64_t *out);
int potts_batch_spins(potts_batch *b, int32_t job, uint8_t *host_out);

/* Device time of the last run in ms (HIP events on the batch's stream), and
 * the launch shapes the tuner chose or read from the cache ("L=<L>:rows=<r>
 * ... <kernel>/q<class>:block=<lanes>,waves/SIMD=<w|auto> ..."). */
double potts_batch_elapsed_ms(const potts_batch *b);
const char *potts_batch_tuning(const potts_batch *b);

/* The digest of the tuned kernels' sources this library was built from: the
 * key under which tuning caches (potts_batch_opts.tune_cache,
 * potts_server_cfg.tune_cache) keep launch shapes.  A cache file is JSON:
 *   {"kernel_hash": "<digest>",
 *    "rows":   {"<strip|packed>/<q class>/<L>": <strip height>, ...},
 *    "shapes": {"<strip|packed>/<q class>": [<lanes 256|128>, <waves/SIMD 0|8>], ...}}
 * q class 0..3 = q <= 16, <= 64, <= 128, <= 256; shapes other than [256, 0]
 * exist for class 0. */
const char *potts_kernel_digest(void);

/* Releases the batch (synchronizes first).  NULL is a no-op. */
void potts_batch_free(potts_batch *b);

/* ---------------------------------------------------------------------------
 * Serving: a server thread admits simulation jobs as they arrive (in arrival
 * order, while a slot is free and the job's lattice and record ring fit in the
 * HBM budget), keeps every admitted lattice and its sweep counter resident on
 * the device, and runs iterations that advance every active job by up to
 * `quantum` sweeps of its current beta point in shared launches (continuous
 * batching): jobs arriving while others run join the next iteration.  Each job
 * gives exactly the bits it gives alone.
 */
typedef struct {
    int64_t hbm_budget;  /* bytes of lattices + record rings held at once (<= 0: 200 GiB) */
    int32_t max_slots;   /* jobs on the device at once (<= 0: 256)              */
    int32_t quantum;     /* sweeps per job per iteration (<= 0: 32)             */
    void *hip_stream;    /* hipStream_t, NULL = the server's own stream         */
    int32_t tune;        /* 1: the first job of a lattice size and q class that
                            the cache does not know has its launch shape timed
                            first, on a throwaway lattice of that size        */
    int32_t _pad;
    const char *tune_cache; /* NULL, or a JSON file of launch shapes (as
                               potts_batch_opts.tune_cache; updated by `tune`) */
} potts_server_cfg;

/* A job: a beta schedule (Sec. 3 protocol), point k run for sweeps[k] sweeps
 * at betas[k] with the configuration carried over.  Point k's summary covers
 * its last ceil(sweeps[k]/2) sweeps (the first half equilibrates).
 * Checkpoints: with `checkpoint` set, the server writes the job's state after
 * every completed point but the last (lattice, sweep counter, next point and
 * the summaries so far; the file is replaced atomically).  A request with
 * `resume_from` naming such a file (same L, q, seed, start and schedule)
 * continues the job from that point: since the random numbers are keyed by
 * (seed, site, sweep), it ends with exactly the bits of an uninterrupted run. */
typedef struct {
    int32_t L, q;            /* L % 16 == 0, 16 <= L <= 65520; 2 <= q <= 256  */
    uint64_t seed;
    int32_t start;           /* potts_start                                   */
    int32_t npoints;         /* 1 .. 4096                                     */
    const double *betas;     /* npoints, copied at submit                     */
    const int64_t *sweeps;   /* npoints, each 1 .. 2^30, copied at submit     */
    int32_t keep_spins;      /* 1: keep the final lattice for collect         */
    int32_t _pad;
    const char *checkpoint;  /* NULL, or the job's checkpoint file (copied)   */
    const char *resume_from; /* NULL, or a checkpoint of this job to continue */
} potts_request;

typedef struct {
    int64_t ticket;
    int32_t L, q, npoints;
    int32_t status;          /* 0, or the negative code that ended the job    */
    int64_t sweeps;          /* sweeps done                                   */
    double t_submit, t_admit, t_done;  /* seconds on the server's clock      */
    int64_t e_sat, nmax;     /* after the last sweep                          */
} potts_served;

typedef struct potts_server potts_server;

int potts_server_start(const potts_server_cfg *cfg, potts_server **out);

/* Queues a job (thread-safe); *ticket identifies it.  Errors: EINVAL (bad
 * fields, or a resume file of another job), EIO (resume file unreadable),
 * ENOMEM (larger than the budget), or the code that stopped a failed
 * server. */
int potts_server_submit(potts_server *srv, const potts_request *req, int64_t *ticket);

/* Up to max tickets of finished jobs not reported before; waits up to
 * timeout_ms (< 0: until one finishes or every job submitted so far is done). */
int potts_server_wait(potts_server *srv, int64_t *tickets, int32_t max, int32_t timeout_ms, int32_t *n);

/* Takes a finished job's results: info, points (npoints summaries, may be
 * NULL) and, when kept, the final lattice (L*L bytes, may be NULL).  Returns
 * the job's status.  Errors: ERANGE (unknown or unfinished ticket). */
int potts_server_collect(potts_server *srv, int64_t ticket, potts_served *info, potts_summary *points,
                         uint8_t *spins);

/* Failure injection for recovery tests, on the host only (nothing on the GPU
 * faults): the job with this ticket, queued or running, ends with status
 * EDEVICE at the first iteration boundary from which its next iteration would
 * run sweep at_sweep (a 0-based sweep index of the job); its device memory is
 * released and the other jobs go on.  Ticket 0 names the next job this
 * server accepts: the failure is attached when the job is submitted, before
 * it can run (a later call with ticket 0 replaces an unclaimed one).
 * Errors: EINVAL (NULL, at_sweep < 0), ERANGE (no such unfinished job). */
int potts_server_inject_fault(potts_server *srv, int64_t ticket, int64_t at_sweep);

/* Waits until every submitted job has finished (timeout_ms < 0: no limit).
 * Errors: ERANGE on time-out, or the code that stopped a failed server. */
int potts_server_drain(potts_server *srv, int32_t timeout_ms);

/* The server's clock (seconds since start) and the number of iterations run. */
double potts_server_now(const potts_server *srv);
int64_t potts_server_iterations(const potts_server *srv);

/* The launch shapes in use: those timed by this server and those read from
 * its cache, as text (as potts_batch_tuning), into out[0..cap) with a
 * terminating NUL (truncated to fit).  Errors: EINVAL. */
int potts_server_tuning(potts_server *srv, char *out, int32_t cap);

/* Finishes every queued and running job, stops the thread and releases the
 * server; returns 0 or the code that failed it.  NULL is a no-op. */
int potts_server_stop(potts_server *srv);

/* Releases the state (synchronizes its stream first).  NULL is a no-op. */
void potts_free(potts_state *s);

/* ---- Simple-cubic lattice (Sec. 7: the checkerboard update in three
 * dimensions, where the lattice still splits into two independent
 * sub-lattices).  The 2D contract lifted to L x L x L sites:
 *   - site (x, y, z) at byte (z L + y) L + x, periodic in all three axes;
 *   - colour (x + y + z) & 1, colour 0 first; six neighbours, so the energy
 *     change of a proposal is dE = n(s) - n(k) in -6..6 and the table holds
 *     thr[d-1] = min(floor(exp(-beta d) 2^32), 2^32 - 1) for d = 1..6 (Eq. 1
 *     with the Metropolis rule of Sec. 3);
 *   - one Philox4x32-10 block per 4-byte row chunk, sweep t and colour c, with
 *     counter (t_lo, ((z L + y) L + x) / 4, t_hi, c + 8) and key (seed_lo,
 *     seed_hi); site x of the chunk takes (w[2b], w[2b+1]), b = (x/2) & 1, as
 *     proposal and acceptance words;
 *   - random start: counter (0, chunk, 0, 10), value floor(w[x & 3] q / 2^32);
 *   - records {e_sat, hist[0..q)} per sweep, e_sat over the 3 L^3 bonds.
 * The state owns its lattice (L^3 bytes, plus a colour-split copy of the same
 * size when that kernel runs), a 4096-slot record ring and a stream.
 * Every call returns 0 or a negative POTTS_E* code (potts_last_error()). */
typedef struct potts3d_state potts3d_state;

/* Creates an L^3 lattice on the current device.  Errors: EINVAL (L < 4,
 * L % 4 != 0, q outside 2..256, bad start, out NULL), ERANGE (L^3/4 >= 2^32),
 * ENOMEM, EDEVICE.  On error *out is NULL. */
int potts3d_init(int32_t L, int32_t q, uint64_t seed, potts_start start, potts3d_state **out);

/* The six-entry Metropolis table above.  Errors: EINVAL (beta < 0, not finite,
 * thr NULL). */
int potts3d_threshold_table(double beta, uint32_t thr[6]);

/* nsweeps full sweeps (colour 0 then colour 1) at beta, each writing its
 * record; asynchronous on the state's stream.  Errors: EINVAL, ERANGE (sweep
 * counter overflow), EDEVICE. */
int potts3d_sweep(potts3d_state *s, double beta, int64_t nsweeps);

/* As potts3d_sweep with a caller-supplied table (host memory, 6 entries). */
int potts3d_sweep_thr(potts3d_state *s, const uint32_t thr[6], int64_t nsweeps);

/* Records of sweeps t0 .. t0+n-1 into out[n*(1+q)] (synchronizes).  Errors:
 * ERANGE if one of them is not (or no longer) in the ring. */
int potts3d_records(potts3d_state *s, int64_t t0, int64_t n, int64_t *out);

/* Measures the current lattice with a kernel of its own (independent of the
 * records; synchronizes). */
int potts3d_observables(potts3d_state *s, potts_obs *out);

/* e, C, V_L, m, chi of the window t0 .. t0+n-1 with N = L^3 (the same
 * definitions and exact moments as potts_stats).  Errors: EINVAL (n outside
 * 1..2^24, bad beta), ERANGE. */
int potts3d_stats(potts3d_state *s, int64_t t0, int64_t n, double beta, potts_summary *out);

/* Copies the lattice (L^3 bytes, layout above) to host memory (synchronizes). */
int potts3d_get_spins(potts3d_state *s, uint8_t *host_out);

/* Kernel choice for later sweeps; every choice gives identical spins and
 * records.  kernel 0: automatic (colour-split when L % 32 == 0, else chunk);
 * 1: colour-split (the state keeps a second L^3-byte copy of the cube split
 * into its two colour planes, allocated on first use, and rebuilds the
 * row-major cube only when it is read); 2: chunk (row-major, any L).  rows:
 * rows of y walked by one colour-split work item, 0 automatic, else an even
 * divisor of L.  Errors: EINVAL (kernel 1 with L % 32 != 0, bad values). */
int potts3d_tune(potts3d_state *s, int32_t kernel, int32_t rows);

/* Sweeps done so far, or -1 for NULL. */
int64_t potts3d_time(const potts3d_state *s);

/* The state's stream (a hipStream_t; NULL for NULL), for callers that order
 * their own work or events after its sweeps. */
void *potts3d_stream(const potts3d_state *s);

/* Releases the state (synchronizes first).  NULL is a no-op. */
void potts3d_free(potts3d_state *s);

/* ---- First and second neighbours on the square lattice (Sec. 7: with
 * second-neighbour couplings the lattice splits into nine independent
 * sub-lattices instead of two).  Contract:
 *   - H = -sum_<ij> delta(s_i, s_j) - j2 sum_<<ij>> delta(s_i, s_j) over the
 *     four nearest (coupling 1) and four diagonal (coupling j2) neighbours;
 *   - L x L periodic, row-major uint8 as the nearest-neighbour lattice,
 *     L % 12 == 0; colour c = 3 (y mod 3) + (x mod 3); one sweep updates
 *     colours 0..8 in turn;
 *   - with d1 = n1(s) - n1(k) and d2 = n2(s) - n2(k) (n1/n2: nearest/diagonal
 *     neighbours equal to a value), the 81-entry table holds at index
 *     (d1 + 4) * 9 + (d2 + 4) the value 2^32 when d1 + j2 d2 <= 0, else
 *     min(floor(exp(-beta (d1 + j2 d2)) 2^32), 2^32 - 1), computed in FP64 on
 *     the host; a move is accepted iff w_acc < entry;
 *   - one Philox4x32-10 block per 6-byte row segment, sweep and colour:
 *     counter (t_lo, y L/6 + x/6, t_hi, 16 + c), key (seed_lo, seed_hi); site
 *     x takes (w[2b], w[2b+1]), b = (x/3) & 1, as proposal and acceptance
 *     words (a segment holds two sites of each colour);
 *   - initial conditions as potts_init;
 *   - records {e1, e2, hist[0..q)} per sweep: satisfied nearest bonds (2N),
 *     satisfied diagonal bonds (2N), populations.
 * The state owns an L*L lattice, a 4096-slot record ring and a stream.  Every
 * call returns 0 or a negative POTTS_E* code (potts_last_error()). */
typedef struct potts_nnn_state potts_nnn_state;

typedef struct {
    int64_t t;                 /* sweeps done                               */
    int64_t e1;                /* satisfied nearest-neighbour bonds         */
    int64_t e2;                /* satisfied diagonal bonds                  */
    int64_t nmax;              /* max_v hist[v]                             */
    int32_t q;
    int32_t L;
    int64_t hist[POTTS_QMAX];  /* valid for v < q                           */
} potts_nnn_obs;

/* Errors: EINVAL (L < 12, L % 12 != 0, q outside 2..256, bad start, out NULL),
 * ERANGE (L*L/4 >= 2^32), ENOMEM, EDEVICE.  On error *out is NULL. */
int potts_nnn_init(int32_t L, int32_t q, uint64_t seed, potts_start start, potts_nnn_state **out);

/* The 81-entry table above.  Errors: EINVAL (beta < 0 or not finite, j2 not
 * finite, thr NULL). */
int potts_nnn_table(double beta, double j2, uint64_t thr[81]);

/* nsweeps sweeps (nine colour passes and the record each) at (beta, j2);
 * asynchronous on the state's stream.  Errors: EINVAL, ERANGE, EDEVICE. */
int potts_nnn_sweep(potts_nnn_state *s, double beta, double j2, int64_t nsweeps);

/* As potts_nnn_sweep with a caller table (host memory, 81 entries <= 2^32). */
int potts_nnn_sweep_thr(potts_nnn_state *s, const uint64_t thr[81], int64_t nsweeps);

/* Records of sweeps t0 .. t0+n-1 into out[n*(2+q)] (synchronizes).  Errors:
 * ERANGE if one of them is not (or no longer) in the ring (the last 4095). */
int potts_nnn_records(potts_nnn_state *s, int64_t t0, int64_t n, int64_t *out);

/* Measures the current lattice (synchronizes). */
int potts_nnn_observables(potts_nnn_state *s, potts_nnn_obs *out);

/* Copies the lattice (L*L bytes, row-major) to host memory (synchronizes). */
int potts_nnn_get_spins(potts_nnn_state *s, uint8_t *host_out);

/* Kernel choice for later sweeps; every choice gives identical spins and
 * records.  0: automatic (1 when L <= 16380, else 2); 1: one launch per row
 * class y mod 3 doing its three colours with rows y-1, y, y+1 staged in LDS;
 * 2: one launch per colour, reading the lattice in place.  Errors: EINVAL
 * (kernel outside 0..2, kernel 1 with L > 16380). */
int potts_nnn_tune(potts_nnn_state *s, int32_t kernel);

/* Sweeps done so far, or -1 for NULL. */
int64_t potts_nnn_time(const potts_nnn_state *s);

/* The state's stream (a hipStream_t; NULL for NULL). */
void *potts_nnn_stream(const potts_nnn_state *s);

/* Releases the state (synchronizes first).  NULL is a no-op. */
void potts_nnn_free(potts_nnn_state *s);

const char *potts_strerror(int code);
const char *potts_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* POTTS_H */
