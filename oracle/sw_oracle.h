/*
 * sw_oracle.h -- CPU oracle for the Swendsen-Wang sweep (TEST INFRASTRUCTURE).
 *
 * This is the plain, sequential, obviously-correct reference that the GPU
 * library is checked against.  It is test infrastructure: only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  The
 * product library never links, loads or calls it, and it includes nothing from
 * the product sources (it carries its own Philox, its own cutoff tables and its
 * own labeling).
 *
 * Method: Komura & Okabe, "GPU-based Swendsen-Wang multi-cluster algorithm for
 * the simulation of two-dimensional classical spin systems" (arXiv:1202.0635).
 *   - Potts Hamiltonian H = -J sum_<ij> (delta(S_i,S_j) - 1), periodic (Sec. 2, Eq. 1)
 *   - CPU SW procedure (i)-(viii): bonds, Hoshen-Kopelman labeling, per-cluster
 *     new value uniform over q (Sec. 2, itemised list)
 *   - proper label = smallest label of the cluster, found by chasing
 *     label[label] (Sec. 2, paragraph after the list)
 *   - clock Hamiltonian H = -J sum S_i.S_j with theta = 2 pi p / q and
 *     Wolff's embedded clusters (Sec. 4, clock-model equation and the
 *     paragraph after it)
 *   - M^2 order parameter (Sec. 4, equation after the moment ratio) and the
 *     moment ratio U = <M^4>/<M^2>^2 (Sec. 4, first equation)
 *
 * Readings fixed where the paper is silent (random numbers, cutoff rounding,
 * the embedded-cluster mirror) form the determinism contract; it is restated
 * in the comments of sw_oracle.c next to each function.
 *
 * Conventions: site i = y*L + x, 0 <= x,y < L; spins are int8 in {0..q-1}
 * (paper's S = k+1); site i owns its right bond (x,y)-(x+1 mod L,y) and its
 * down bond (x,y)-(x,y+1 mod L).  Bond arrays are one uint8 (0/1) per site.
 */
#ifndef SW_ORACLE_H
#define SW_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_POTTS = 0, OR_CLOCK = 1 };
enum { OR_P_BOND_HI = 0, OR_P_BOND_LO = 1, OR_P_CLUSTER = 2, OR_P_MIRROR = 3, OR_P_INIT = 4 };

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Draw of the contract: key = seed, counter = (c0, t mod 2^32, purpose, t >> 32). */
void or_draw(uint64_t seed, uint32_t c0, uint64_t t, uint32_t purpose, uint32_t out[4]);
/* Map a uniform 32-bit word to {0..q-1}: (w*q) >> 32. */
uint32_t or_qmap(uint32_t w, uint32_t q);

/* Cutoff table.  Potts: q*q entries C[a*q+b]; clock: q*q*q entries C[(m*q+a)*q+b].
 * Returns the number of entries written, or -1 on invalid parameters. */
int or_table_size(int model, int q);
int or_cutoffs(int model, int q, double T, double J, uint32_t* table);
/* The projected product P(a,b,m) of the clock embedding (for inspection). */
double or_clock_projection(int q, int a, int b, int m);

void or_init(int L, int q, uint64_t seed, int8_t* spins);
int or_mirror(int q, uint64_t seed, uint64_t t);
void or_bonds(int L, int q, int model, const uint32_t* table, uint64_t seed, uint64_t t,
              const int8_t* spins, uint8_t* bond_r, uint8_t* bond_d);
/* The bonds owned by the n sites sites[k] (row-major indices), from the
 * whole state spins: bond_r[k], bond_d[k]. */
void or_bonds_at(int L, int q, int model, const uint32_t* table, uint64_t seed, uint64_t t,
                 const int8_t* spins, int64_t n, const int64_t* sites, uint8_t* bond_r, uint8_t* bond_d);
void or_label(int L, const uint8_t* bond_r, const uint8_t* bond_d, int32_t* label);
void or_flip(int L, int q, int model, uint64_t seed, uint64_t t, const int32_t* label,
             int8_t* spins);
/* The flip of n single sites: site k has canonical label root[k] and old
 * value old[k]; out[k] receives its new value. */
void or_flip_at(int q, int model, uint64_t seed, uint64_t t, int64_t n, const int32_t* root,
                const int8_t* old, int8_t* out);
/* One full sweep t: bonds, labels, flip.  label (N int32) receives the
 * canonical labels; bond_r/bond_d (N uint8) the bonds.  Returns the number of
 * clusters. */
int64_t or_sweep(int L, int q, int model, const uint32_t* table, uint64_t seed, uint64_t t,
                 int8_t* spins, uint8_t* bond_r, uint8_t* bond_d, int32_t* label);

/* Integer counts of a state: hist[k] (k<q) and pair_hist[d] over the 2N owned
 * bonds, d = (s_j - s_i) mod q. */
void or_counts(int L, int q, const int8_t* spins, int64_t* hist, int64_t* pair_hist);
/* Correlation counts at distance r: the histogram of (s_j - s_i) mod q over
 * the 2N pairs j = i + r (x direction) and j = i + r (y direction), periodic;
 * and G(r) from them (mean of cos(theta_j - theta_i)). */
void or_corr_counts(int L, int q, const int8_t* spins, int r, int64_t* corr_hist);
double or_corr_g(int L, int q, const int64_t* corr_hist);
/* Observables from counts: energy per site and M^2 / N^2 (Potts order
 * parameter of the paper, or |M|^2/N^2 for the clock model). */
void or_observables(int L, int q, int model, double J, const int64_t* hist,
                    const int64_t* pair_hist, double* e_per_site, double* m2);

/* Run a chain from the Philox random start: n_therm unmeasured sweeps, then
 * n_meas sweeps each followed by a measurement written to e[k], m2[k].
 * spins (N int8) holds the final state on return.  Returns 0, or -1. */
int or_run(int L, int q, int model, double T, double J, uint64_t seed, int64_t n_therm,
           int64_t n_meas, int8_t* spins, double* e, double* m2);

/* One sweep at sweep index t from the state s0, repeated for seeds
 * seed0..seed0+nseeds-1; counts[state] is incremented for the resulting state,
 * state = sum_i s_i q^i (requires q^N <= 2^31).  For transition-matrix tests on
 * tiny lattices. */
int or_transition_counts(int L, int q, int model, double T, double J, const int8_t* s0,
                         uint64_t t, uint64_t seed0, int64_t nseeds, int64_t* counts);

/* SplitMix64 finaliser and the order-independent state hashes. */
uint64_t or_mix64(uint64_t z);
uint64_t or_hash_spins(int64_t n, const int8_t* spins);
uint64_t or_hash_labels(int64_t n, const int32_t* label);

#ifdef __cplusplus
}
#endif
#endif
