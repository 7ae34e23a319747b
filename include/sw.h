/*
 * sw.h -- C-ABI of libswmc: the Swendsen-Wang multi-cluster sweep for 2D
 * q-state Potts and q-state clock models on AMD Instinct MI355X (gfx950).
 *
 * Method: Komura & Okabe, "GPU-based Swendsen-Wang multi-cluster algorithm
 * for the simulation of two-dimensional classical spin systems"
 * (arXiv:1202.0635).  One sweep has the three steps of Sec. 2:
 *   (1) Fortuin-Kasteleyn bond activation between neighbours,
 *   (2) connected-component labeling of the bond graph,
 *   (3) a new random value (Potts) or a random reflection (clock, Wolff's
 *       embedded cluster, Sec. 4) for every cluster.
 *
 * Every call returns an sw_status (0 = SW_OK, negative = error) and never
 * throws.  Invalid parameters are rejected before any device work.  A device
 * error is sticky: afterwards every call on that context returns SW_ESTATE
 * until sw_free.  sw_last_error() gives a thread-local detail string for the
 * last failing call of the calling thread.
 *
 * Determinism: the chain is a pure function of (sw_lattice, number of sweeps).
 * All random numbers are Philox4x32-10 draws keyed by the seed, with the
 * counter (index, sweep mod 2^32, purpose, sweep >> 32); bond thresholds come
 * from a host FP64 table as uint32 cutoffs; the canonical label of a cluster
 * is its smallest site index (Sec. 2: the proper label is the smallest).
 * Results do not depend on tiling, batching or scheduling.
 *
 * Conventions: site i = y*L + x; spins are int8 in {0..q-1} (the paper's
 * S = k+1 for Potts, angle 2 pi k / q for the clock model); site i owns its
 * right bond to (x+1 mod L, y) and its down bond to (x, y+1 mod L).  Periodic
 * boundaries (Sec. 2).
 *
 * Concurrency: one context per stream; a context is not thread-safe, distinct
 * contexts are independent.
 */
#ifndef SW_H
#define SW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SW_OK = 0,
    SW_EINVAL = -1,   /* invalid argument (checked before any device work) */
    SW_ENOMEM = -2,   /* device memory: allocation failed or caller buffer too small */
    SW_EDEVICE = -3,  /* a HIP runtime call failed; the context becomes unusable */
    SW_ESTATE = -4,   /* the context had a device error earlier, or a call came out of order */
    SW_EBUDGET = -5,  /* (server) a request does not fit the memory budget */
    SW_EBUSY = -6     /* (server) no free slot or result not ready */
} sw_status;

typedef enum { SW_POTTS = 0, SW_CLOCK = 1 } sw_model;

/* flags of sw_sweep */
enum {
    SW_MEASURE = 1u, /* accumulate E, M^2, M^4 after every sweep of this call */
    SW_VERIFY = 2u,  /* also store the canonical labels of the last sweep */
    SW_PROFILE = 4u, /* time every kernel launch with HIP events (read by sw_profile_read) */
    SW_NO_GRAPH = 8u, /* batches: launch the kernels directly instead of replaying the captured sweep */
    SW_HASH = 16u     /* record the state hashes of every sweep (read by sw_read_hashes) */
};

/* One lattice.  Potts: H = -J sum_<ij> (delta(S_i,S_j) - 1) (Sec. 2, Eq. 1);
 * clock: H = -J sum_<ij> S_i . S_j with S = (cos 2 pi k/q, sin 2 pi k/q) (Sec. 4).
 * Valid: 2 <= q <= 32, model in {SW_POTTS, SW_CLOCK}, 0 < T, 0 < J (finite),
 * reserved 0, and 2 <= L <= 65535 for a single lattice (sw_init; site indices
 * below 2^32), 2 <= L <= 46340 for batches, the server, sw_sweep_static and
 * the label-equivalence labelers (site indices below 2^31). */
typedef struct {
    int32_t L, q, model, reserved;
    double T, J;
    uint64_t seed;
} sw_lattice;

/* Observables.  Integer fields are exact; doubles are derived on the host in
 * FP64 in a fixed order.  e_per_site = H / N.  m2 = M^2 / N^2 with the Potts
 * order parameter M^2 = (q sum_k n[k]^2 - N^2)/(q-1) (Sec. 4, equation after
 * the moment ratio), or |M|^2 / N^2 for the clock model.  mean_* are running
 * averages over the sweeps measured so far (SW_MEASURE); m4 is (M^2)^2 and
 * binder_u = <M^4>/<M^2>^2 is the moment ratio of Sec. 4. */
typedef struct {
    uint64_t sweeps_done; /* sweep index t of the current state */
    uint64_t samples;     /* number of measured sweeps accumulated */
    int64_t hist[32];     /* n[k], number of sites in state k (k < q) */
    int64_t pair_hist[32];/* owned bonds (2N) by (s_j - s_i) mod q */
    double e_per_site, m2;
    double mean_e, mean_m2, mean_m4, binder_u;
    /* Clock model only (zero for Potts): the correlation function of Sec. 4,
     * G(r) = <S_i^x S_{i+r}^x + S_i^y S_{i+r}^y>, at r = L/4 and r = L/2 (integer
     * division).  corr_hist[0] and corr_hist[1] count the 2N pairs (i, i + r x)
     * and (i, i + r y) (periodic) by (s_j - s_i) mod q, for r = L/4 and L/2;
     * g_quarter and g_half are G of the current state (FP64 from the counts);
     * mean_g_* are running averages over the measured sweeps and
     * corr_ratio = mean_g_half / mean_g_quarter is the ratio R(T) (0 while
     * mean_g_quarter is 0). */
    int64_t corr_hist[2][32];
    double g_quarter, g_half;
    double mean_g_quarter, mean_g_half, corr_ratio;
    /* |M| / N = sqrt(m2) of the current state. */
    double absm;
    /* Order-independent fingerprints, computed on the device:
     * hash_spins  = sum_i mix64((i << 8) | s_i) mod 2^64 of the current state;
     * hash_labels = sum_i mix64((i << 32) | l_i) mod 2^64 of the canonical
     *               labels l_i of the last sweep run with SW_VERIFY (0 if none);
     * mix64 is the SplitMix64 output function (Steele, Lea & Flood 2014).
     * Equal states (labels) give equal hashes; the hashes let a long chain be
     * compared with the oracle sweep by sweep without whole-state copies. */
    uint64_t hash_spins, hash_labels;
} sw_obs;

typedef struct sw_ctx sw_ctx;

/* Device bytes needed for one lattice (arena for sw_init); 0 if *p is invalid. */
size_t sw_state_bytes(const sw_lattice* p);

/* Create a context and the random start (s_i = qmap(Philox(i, 0, init)), t = 0).
 * dev_mem: caller-owned device buffer of at least sw_state_bytes(p) bytes,
 *          256-byte aligned, which the context uses and never frees; or NULL,
 *          in which case the library allocates (and sw_free releases) it.
 * stream:  hipStream_t (NULL = the null stream); every kernel of this context
 *          runs on it, and calls that return data synchronise it.
 * Errors: SW_EINVAL (bad parameters, unaligned or short buffer), SW_ENOMEM,
 *         SW_EDEVICE.  On error *out is NULL. */
int sw_init(const sw_lattice* p, void* dev_mem, size_t bytes, void* stream, sw_ctx** out);

/* Run nsweeps >= 0 sweeps (Sec. 2 steps (1)-(3), Sec. 3 for the GPU), enqueued
 * asynchronously on the stream.  flags: SW_MEASURE | SW_VERIFY | SW_PROFILE |
 * SW_HASH.  With SW_MEASURE (SW_HASH) the call synchronises every 1024 sweeps
 * and at its end to fold the per-sweep counts into the running averages (to
 * move the hashes to the host).  A kernel that finds the label forest broken
 * (a walk longer than its node count) records it on the device; the next
 * synchronising call then returns SW_EDEVICE and the context becomes sticky. */
int sw_sweep(sw_ctx* c, int32_t nsweeps, uint32_t flags);

/* Observables of the current state plus the running averages (synchronises). */
int sw_measure(sw_ctx* c, sw_obs* out);

/* Per-sweep state hashes of the sweeps run with SW_HASH since the last read,
 * oldest first: record k is out[3k] = the sweep index t of the state after
 * that sweep (sweeps_done), out[3k+1] = its hash_spins and out[3k+2] the
 * hash_labels of that sweep's canonical labels (definitions at sw_obs).  The
 * canonical labels (Sec. 2: the proper label of a cluster is its smallest
 * site index) are read from the label forest after the sweep's border merge,
 * so every sweep of a multi-sweep call is covered.  Moves up to cap records
 * to out (3 * cap words) and sets *n; records not moved stay for the next
 * read.  Synchronises. */
int sw_read_hashes(sw_ctx* c, uint64_t* out, size_t cap, size_t* n);

/* Synchronous copies to host memory.  n must equal N = L*L (SW_EINVAL otherwise).
 * sw_read_labels returns the canonical labels (smallest site index of the
 * cluster) of the last sweep run with SW_VERIFY (SW_ESTATE if there was none).
 * sw_read_bonds returns one byte (0/1) per site for the right and down bonds of
 * the last sweep. */
int sw_read_spins(sw_ctx* c, int8_t* host, size_t n);
int sw_read_labels(sw_ctx* c, int32_t* host, size_t n);
int sw_read_bonds(sw_ctx* c, uint8_t* host_right, uint8_t* host_down, size_t n);

/* Replace the state (restore / tests): spins host[n] with values < q
 * (SW_EINVAL otherwise) and the sweep index t.  Synchronous. */
int sw_write_spins(sw_ctx* c, const int8_t* host, size_t n, uint64_t t);

/* Device address of the spin array (int8[N], row-major) owned by the context. */
int sw_device_spins(sw_ctx* c, void** dev_ptr);

/* Host-only: the uint32 cutoff table of the bond rule (Sec. 2 step (ii); Sec. 4
 * embedded cluster).  Potts: q*q entries C[a*q+b]; clock: q^3 entries
 * C[(m*q+a)*q+b].  n must equal that size.  Needs no GPU. */
int sw_cutoff_table(const sw_lattice* p, uint32_t* out, size_t n);

/* Per-kernel timing of the sweeps run with SW_PROFILE since the last read:
 * names[k] (static strings), launches[k], total_ms[k] for k < *nk (at most
 * cap).  Synchronises.  Resets the accumulators. */
int sw_profile_read(sw_ctx* c, const char** names, int64_t* launches, double* total_ms,
                    int32_t cap, int32_t* nk);

/* Waves per 64 x 64 tile of the bond kernel: 4 (16 rows each) or 8 (8 rows
 * each).  The default is 8 for lattices of fewer than 3072 tiles (L <= 3520),
 * where 4-wave workgroups leave the chip's SIMDs short of waves, else 4.
 * Other values: SW_EINVAL.  Results do not depend on it; only the time does. */
int sw_set_tile_waves(sw_ctx* c, int32_t waves);
/* Autotuner: times `sweeps` sweeps with 4 and with 8 waves per tile from the
 * current state (three rounds, each choice's fastest counts), restores the
 * state (spins and sweep index) after each, keeps the faster and returns it in
 * *waves.  The choice is remembered per (architecture, ceil(log2 L), model, q)
 * for the process, and across processes in the file named by the environment
 * variable SWMC_TUNE_CACHE if set; a remembered choice is applied without
 * timing.  Allocates a temporary snapshot buffer. */
int sw_tune(sw_ctx* c, int32_t sweeps, int32_t* waves);

/* The cluster labeler (Sec. 3).  SW_LABEL_UNION_FIND (default): tile-local
 * union-find in LDS, then lock-free unions across tile borders.
 * SW_LABEL_HAWICK and SW_LABEL_KALENTEV: the two label-equivalence labelers the
 * paper adapts (Sec. 3; Hawick et al. with the temporary array and atomic
 * minimum, Kalentev et al. with one array and no atomics), iterated until a
 * scan changes nothing, with the host reading a flag after every iteration as
 * in the paper.  Kept as an ablation: canonical labels are unique, so every
 * labeler gives the same chain; only the time differs.  Single-lattice contexts
 * only; other values: SW_EINVAL. */
enum { SW_LABEL_UNION_FIND = 0, SW_LABEL_HAWICK = 1, SW_LABEL_KALENTEV = 2 };
int sw_set_labeler(sw_ctx* c, int32_t labeler);
/* Label-equivalence iterations run since the context was made (scan passes,
 * the last of each sweep included) and the sweeps they served. */
int sw_labeler_stats(sw_ctx* c, uint64_t* iterations, uint64_t* sweeps);

void sw_free(sw_ctx* c);
const char* sw_strerror(int status);
const char* sw_last_error(void);

/* ---------------------------------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * sw_sweep_static runs nsweeps >= 0 sweeps of the lattice *p, as sw_sweep
 * does, without a context and without allocating anything: no hipMalloc, no
 * hipFree, no stream or event creation.  The label forest, bond masks,
 * border records and control block live in one static device buffer of the
 * library, SW_STATIC_SCRATCH_BYTES bytes on each GPU it runs on (sized for
 * L <= SW_STATIC_MAX_L; held until the process ends).
 *   spins:  device int8[L*L] (caller-owned, 16-byte aligned), the state at
 *           sweep index t on entry; replaced in place by the state at sweep
 *           t + nsweeps.
 *   table:  device copy of the cutoff table of *p (sw_cutoff_table).
 *   labels: device int32[L*L] (16-byte aligned) or NULL; if given (nsweeps >= 1), receives the
 *           canonical labels (smallest site index of the cluster) of the
 *           last sweep.
 *   fault:  device uint32 or NULL; if given, receives 0, or the nonzero
 *           fault bits of a kernel that found the label forest broken.
 * Every kernel is enqueued on stream (NULL = the null stream); the call
 * returns without waiting.  The results equal sw_init + sw_write_spins(t) +
 * sw_sweep(nsweeps) bit for bit.  Errors: SW_EINVAL (invalid lattice,
 * L > SW_STATIC_MAX_L, null spins or table, misaligned pointers, labels with
 * nsweeps = 0) before
 * any device work; SW_EDEVICE if a launch fails.
 * All calls on one GPU share its buffer: calls that overlap in time on one
 * GPU (different streams, or threads) race and corrupt each other; serialise
 * them, e.g. on one stream. */
#define SW_STATIC_MAX_L 1024
#define SW_STATIC_SCRATCH_BYTES 4735232u
int sw_sweep_static(const sw_lattice* p, int8_t* spins, uint64_t t, int32_t nsweeps, const uint32_t* table,
                    int32_t* labels, uint32_t* fault, void* stream);

/* ---------------------------------------------------------------------------
 * Batches: n independent lattices (replicas of any L, q, model, T, seed) swept
 * together.  Every phase of a sweep (Sec. 2 steps (1)-(3)) is one launch over
 * the workgroups of all replicas; one sweep's launches are captured once in a
 * hipGraph and replayed: a call of n sweeps is one graph launch for up to 512
 * sweeps (a run of n sweeps captured once, the last four run lengths kept).
 * Each replica's chain is bit-identical to the same lattice run alone through
 * sw_init/sw_sweep.
 * ------------------------------------------------------------------------- */
typedef struct sw_batch sw_batch;

/* Device bytes for the batch arena (replica states + launch maps); 0 if any
 * lattice is invalid or n is not in [1, 65535]. */
size_t sw_batch_bytes(const sw_lattice* ps, int32_t n);
/* ps[n] as in sw_init; dev_mem caller-owned (256-byte aligned, at least
 * sw_batch_bytes) or NULL (library-owned).  Random start for every replica. */
int sw_batch_init(const sw_lattice* ps, int32_t n, void* dev_mem, size_t bytes, void* stream, sw_batch** out);
/* nsweeps sweeps of every replica; flags SW_MEASURE | SW_VERIFY | SW_PROFILE |
 * SW_HASH | SW_NO_GRAPH (the graph is used only without SW_MEASURE, SW_HASH
 * and SW_PROFILE). */
int sw_batch_sweep(sw_batch* b, int32_t nsweeps, uint32_t flags);
/* Per replica, as sw_measure / sw_read_spins / sw_read_labels (synchronous). */
int sw_batch_measure(sw_batch* b, int32_t replica, sw_obs* out);
int sw_batch_read_spins(sw_batch* b, int32_t replica, int8_t* host, size_t n);
int sw_batch_read_labels(sw_batch* b, int32_t replica, int32_t* host, size_t n);
/* As sw_read_hashes, for one replica (the sweeps run with SW_HASH). */
int sw_batch_read_hashes(sw_batch* b, int32_t replica, uint64_t* out, size_t cap, size_t* n);
int32_t sw_batch_size(sw_batch* b);
/* Merge schedule (as sw_set_schedule of the paper's one-level design: 1 = one
 * device-wide border kernel; 2 or 4 = the inner borders of blocks of that
 * many tiles per side first joined in LDS) and waves per tile of the batched
 * bond kernel (4 or 8).  Other values: SW_EINVAL.  Results do not depend on
 * either; only the time does. */
int sw_batch_set_schedule(sw_batch* b, int32_t merge_tiles);
int sw_batch_set_tile_waves(sw_batch* b, int32_t waves);
/* Autotuner: times a captured run of `sweeps` sweeps for every pair of waves
 * per tile {4, 8} and merge schedule {1, 2, 4} from the same saved state,
 * restores the state after each, keeps the fastest pair and returns it in
 * *merge_tiles and *waves (may be NULL).  Choices are remembered per key
 * (architecture, total sites bucket, largest L bucket, models present) for the
 * process, and across processes in the file named by the environment variable
 * SWMC_TUNE_CACHE if set; a remembered choice is applied without timing.
 * Allocates a temporary snapshot buffer. */
int sw_batch_tune(sw_batch* b, int32_t sweeps, int32_t* merge_tiles, int32_t* waves);
int sw_batch_profile_read(sw_batch* b, const char** names, int64_t* launches, double* total_ms, int32_t cap,
                          int32_t* nk);
void sw_batch_free(sw_batch* b);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of simulation requests.  A request is one
 * lattice and a sweep count.  Requests wait in arrival order; at every step
 * the server admits waiting requests while their state fits the device-memory
 * budget and a slot is free (a request that cannot fit waits at the head of
 * the queue), then runs sweeps_per_step sweeps over every active lattice as
 * one batched launch per phase (a lattice that reaches its sweep count sits
 * the rest of the step out), then retires the finished ones: their final
 * observables and spin hash become results and their memory is freed.  Each
 * result is identical to running that lattice alone.  The caller drives the
 * server (submit / step / poll); a server is not thread-safe.
 * ------------------------------------------------------------------------- */
typedef struct sw_server sw_server;

typedef struct {
    sw_lattice lattice;
    int64_t sweeps;   /* sweeps from the random start, >= 1 */
    uint64_t tag;     /* caller's id, returned with the result */
    double t_arrival; /* arrival time on the server clock (sw_server_now); latency counts from it */
} sw_request;

typedef struct {
    uint64_t tag;
    int32_t status;     /* SW_OK, or SW_EBUDGET: the request can never fit the budget */
    int32_t reserved;
    sw_obs obs;         /* observables of the final state (obs.sweeps_done == sweeps) */
    uint64_t spin_hash; /* sum over sites of SplitMix64-finalised ((i << 8) | s_i), mod 2^64 */
    double t_arrival, t_admit, t_done;
} sw_result;

typedef struct {
    int64_t submitted, waiting, active, completed, rejected, steps;
    int64_t spin_updates; /* sum of L^2 * sweeps over completed requests */
    uint64_t budget_bytes, used_bytes;
} sw_server_stats;

/* budget_bytes: device memory for lattice states (allocated once here);
 * max_slots >= 1 lattices at a time; sweeps_per_step >= 1. */
int sw_server_create(uint64_t budget_bytes, int32_t max_slots, int32_t sweeps_per_step, void* stream,
                     sw_server** out);
double sw_server_now(sw_server* s);
/* Queue a request (SW_EINVAL for an invalid lattice or sweeps < 1; a request
 * larger than the whole budget is completed at once with status SW_EBUDGET). */
int sw_server_submit(sw_server* s, const sw_request* req);
/* Admit, run one step, retire; synchronous.  *active = lattices that ran. */
int sw_server_step(sw_server* s, int32_t* active);
/* Move up to cap finished results to out[]; *n = how many. */
int sw_server_poll(sw_server* s, sw_result* out, int32_t cap, int32_t* n);
int sw_server_stats_read(sw_server* s, sw_server_stats* out);
void sw_server_destroy(sw_server* s);

#ifdef __cplusplus
}
#endif
#endif /* SW_H */
