/*
 * sw_oracle.c -- CPU oracle for the Swendsen-Wang sweep (TEST INFRASTRUCTURE).
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this file's library.  It is written to be read against the paper
 * (Komura & Okabe, arXiv:1202.0635), not to be fast: one site at a time, in
 * the order of the CPU procedure of Sec. 2, with the Hoshen-Kopelman labeling
 * the paper names for the CPU.
 *
 * Determinism contract (readings of what the paper leaves open; the GPU
 * library implements the same contract independently):
 *   R1  Random numbers: Philox4x32-10 keyed by the 64-bit seed (low word
 *       first), counter (c0, t mod 2^32, purpose, t >> 32).  The paper used a
 *       linear congruential generator (Sec. 3, last paragraph); a counter-based
 *       generator makes every draw a pure function of (seed, site, sweep).
 *   R2  Bond uniforms are 32-bit: u = (hi << 24) | lo.  The high bytes come
 *       from one draw per column and group of eight rows (purpose 0,
 *       c0 = (y div 8)*L + x): word k serves rows 8*(y div 8) + 2k and
 *       8*(y div 8) + 2k + 1; its bytes, most significant first, are the right
 *       and the down bond of the first of these rows, then the right and the
 *       down bond of the second.  The low 24 bits come from a draw per site
 *       (purpose 1, c0 = i): word 0 for the right bond, word 1 for the down
 *       bond.
 *   R3  A bond is active iff u < C(s_i, s_j), with the cutoff
 *       C = floor(2^32 * p) from a host FP64 table, p = 1 - exp(-x) evaluated
 *       as -expm1(-x), clamped to 2^32-1.  Potts: x = J/T for equal spins and
 *       no bond otherwise (Sec. 2, step (ii)).  Clock: x = 2 J P / T when
 *       P > 0, else no bond, with P the product of the two spins' projections
 *       on the mirror normal (Sec. 4, embedded cluster).
 *   R4  Clock mirror: one mirror index m per sweep, m = qmap(purpose 3,
 *       c0 = 0); the reflection maps k to (m - k) mod q, i.e. the projection
 *       direction has angle phi = pi m / q + pi / 2, and
 *       P(a,b,m) = [cos(2pi(a-b)/q) - cos(2pi(a+b-m)/q)] / 2.
 *   R5  Canonical label = smallest site index of the cluster (the paper's
 *       "proper label" is the smallest label, Sec. 2).
 *   R6  Flip: each cluster draws at its canonical label rho (purpose 2).
 *       Potts q >= 3: W = word 0 of the draw with c0 = rho; new value qmap(W),
 *       uniform over all q values, the old value included (Sec. 2, step
 *       (vi)).  The two-outcome cases take one bit B: bit (rho mod 128) of the
 *       draw with c0 = rho div 128 (word k of a draw holds bits 32k to
 *       32k + 31, least significant first).  Potts q = 2: new value B (the
 *       same map, qmap(B * 2^31, 2) = B).  Clock: the cluster is reflected
 *       iff B = 1 (probability 1/2).
 *   R7  Random start: s_i = qmap(word 0 of purpose 4, c0 = i, t = 0).
 *   R8  qmap(w) = (w * q) >> 32 in 64-bit arithmetic.
 */
#include "sw_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11, Sec. 5: the Philox S-box uses two   */
/* 32x32->64 multiplications per round; the key is bumped by the Weyl      */
/* constants between rounds).                                               */
/* ------------------------------------------------------------------ */
#define OR_PHILOX_M0 0xD2511F53u
#define OR_PHILOX_M1 0xCD9E8D57u
#define OR_PHILOX_W0 0x9E3779B9u
#define OR_PHILOX_W1 0xBB67AE85u

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += OR_PHILOX_W0;
            k1 += OR_PHILOX_W1;
        }
        uint64_t prod_a = (uint64_t)OR_PHILOX_M0 * (uint64_t)x0;
        uint64_t prod_b = (uint64_t)OR_PHILOX_M1 * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(prod_b >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)prod_b;
        uint32_t y2 = (uint32_t)(prod_a >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)prod_a;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void or_draw(uint64_t seed, uint32_t c0, uint64_t t, uint32_t purpose, uint32_t out[4]) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {c0, (uint32_t)t, purpose, (uint32_t)(t >> 32)};
    or_philox4x32_10(ctr, key, out);
}

uint32_t or_qmap(uint32_t w, uint32_t q) {
    return (uint32_t)(((uint64_t)w * (uint64_t)q) >> 32);
}

/* ------------------------------------------------------------------ */
/* Parameters and cutoff tables (R3, R4).                                   */
/* ------------------------------------------------------------------ */
static int params_ok(int L, int q, int model) {
    if (L < 2 || L > 46340) return 0;
    if (q < 2 || q > 32) return 0;
    if (model != OR_POTTS && model != OR_CLOCK) return 0;
    return 1;
}

/* cos and sin of 2 pi n / q; angles that are multiples of 30 degrees with a
 * rational cosine (or sine) are returned exactly. */
static double cos_turn(int n, int q) {
    n = ((n % q) + q) % q;
    if ((12 * n) % q == 0) {
        switch ((12 * n) / q) {
            case 0: return 1.0;
            case 2: return 0.5;
            case 3: return 0.0;
            case 4: return -0.5;
            case 6: return -1.0;
            case 8: return -0.5;
            case 9: return 0.0;
            case 10: return 0.5;
            default: break;
        }
    }
    return cos(2.0 * M_PI * (double)n / (double)q);
}

static double sin_turn(int n, int q) {
    n = ((n % q) + q) % q;
    if ((12 * n) % q == 0) {
        switch ((12 * n) / q) {
            case 0: return 0.0;
            case 1: return 0.5;
            case 3: return 1.0;
            case 5: return 0.5;
            case 6: return 0.0;
            case 7: return -0.5;
            case 9: return -1.0;
            case 11: return -0.5;
            default: break;
        }
    }
    return sin(2.0 * M_PI * (double)n / (double)q);
}

/* floor(2^32 * (1 - exp(-x))), clamped to the uint32 range. */
static uint32_t cutoff_of(double x) {
    double p = -expm1(-x);
    double c = floor(ldexp(p, 32));
    if (c >= 4294967295.0) return 0xFFFFFFFFu;
    if (c <= 0.0) return 0u;
    return (uint32_t)c;
}

double or_clock_projection(int q, int a, int b, int m) {
    return 0.5 * (cos_turn(a - b, q) - cos_turn(a + b - m, q));
}

int or_table_size(int model, int q) {
    if (q < 2 || q > 32) return -1;
    if (model == OR_POTTS) return q * q;
    if (model == OR_CLOCK) return q * q * q;
    return -1;
}

int or_cutoffs(int model, int q, double T, double J, uint32_t* table) {
    if (!(T > 0.0) || !(J > 0.0) || !isfinite(T) || !isfinite(J)) return -1;
    int n = or_table_size(model, q);
    if (n < 0) return -1;
    if (model == OR_POTTS) {
        /* Sec. 2, step (ii): equal neighbours bond with p = 1 - exp(-J/T). */
        uint32_t c_eq = cutoff_of(J / T);
        for (int a = 0; a < q; ++a)
            for (int b = 0; b < q; ++b) table[a * q + b] = (a == b) ? c_eq : 0u;
    } else {
        /* Embedded Ising couplings J |S_a.r| |S_b.r|: bond with
         * p = 1 - exp(-2 J P / T) when the projections agree in sign (P > 0). */
        for (int m = 0; m < q; ++m)
            for (int a = 0; a < q; ++a)
                for (int b = 0; b < q; ++b) {
                    double P = or_clock_projection(q, a, b, m);
                    table[(m * q + a) * q + b] = (P > 0.0) ? cutoff_of(2.0 * J * P / T) : 0u;
                }
    }
    return n;
}

/* ------------------------------------------------------------------ */
/* Random start (R7) and mirror (R4).                                       */
/* ------------------------------------------------------------------ */
void or_init(int L, int q, uint64_t seed, int8_t* spins) {
    int64_t N = (int64_t)L * L;
    for (int64_t i = 0; i < N; ++i) {
        uint32_t w[4];
        or_draw(seed, (uint32_t)i, 0, OR_P_INIT, w);
        spins[i] = (int8_t)or_qmap(w[0], (uint32_t)q);
    }
}

int or_mirror(int q, uint64_t seed, uint64_t t) {
    uint32_t w[4];
    or_draw(seed, 0u, t, OR_P_MIRROR, w);
    return (int)or_qmap(w[0], (uint32_t)q);
}

/* ------------------------------------------------------------------ */
/* Step 1: active bonds, Sec. 2 steps (i)-(iii).                            */
/* ------------------------------------------------------------------ */
/* The two bonds owned by site (y, x): to its right and to its lower
 * neighbour.  C is the cutoff slice of this sweep (R2, R3). */
static void bond_site(int L, int q, const uint32_t* C, uint64_t seed, uint64_t t, const int8_t* spins,
                      int y, int x, uint8_t* br, uint8_t* bd) {
    int64_t i = (int64_t)y * L + x;
    int64_t j_right = (int64_t)y * L + (x + 1) % L;
    int64_t j_down = (int64_t)((y + 1) % L) * L + x;
    uint32_t w_hi[4], w_lo[4];
    or_draw(seed, (uint32_t)((int64_t)(y / 8) * L + x), t, OR_P_BOND_HI, w_hi);
    or_draw(seed, (uint32_t)i, t, OR_P_BOND_LO, w_lo);
    uint32_t word = w_hi[(y % 8) / 2];
    int shift = (y % 2 == 0) ? 16 : 0; /* this row's two bytes */
    uint32_t hi_right = (word >> (shift + 8)) & 0xFFu;
    uint32_t hi_down = (word >> shift) & 0xFFu;
    uint32_t u_right = (hi_right << 24) | (w_lo[0] & 0x00FFFFFFu);
    uint32_t u_down = (hi_down << 24) | (w_lo[1] & 0x00FFFFFFu);
    int a = spins[i];
    *br = (uint8_t)(u_right < C[a * q + spins[j_right]]);
    *bd = (uint8_t)(u_down < C[a * q + spins[j_down]]);
}

static const uint32_t* cutoff_slice(int q, int model, const uint32_t* table, uint64_t seed, uint64_t t) {
    int m = (model == OR_CLOCK) ? or_mirror(q, seed, t) : 0;
    return (model == OR_CLOCK) ? table + (size_t)m * q * q : table;
}

void or_bonds(int L, int q, int model, const uint32_t* table, uint64_t seed, uint64_t t,
              const int8_t* spins, uint8_t* bond_r, uint8_t* bond_d) {
    const uint32_t* C = cutoff_slice(q, model, table, seed, t);
    for (int y = 0; y < L; ++y) {
        for (int x = 0; x < L; ++x) {
            int64_t i = (int64_t)y * L + x;
            bond_site(L, q, C, seed, t, spins, y, x, &bond_r[i], &bond_d[i]);
        }
    }
}

void or_bonds_at(int L, int q, int model, const uint32_t* table, uint64_t seed, uint64_t t,
                 const int8_t* spins, int64_t n, const int64_t* sites, uint8_t* bond_r, uint8_t* bond_d) {
    const uint32_t* C = cutoff_slice(q, model, table, seed, t);
    for (int64_t k = 0; k < n; ++k)
        bond_site(L, q, C, seed, t, spins, (int)(sites[k] / L), (int)(sites[k] % L), &bond_r[k], &bond_d[k]);
}

/* ------------------------------------------------------------------ */
/* Step 2: Hoshen-Kopelman labeling (Sec. 2).  label[] holds site indices;   */
/* a label's proper label is found by evaluating label[label] repeatedly,   */
/* and the proper label of a cluster is its smallest one (R5).              */
/* ------------------------------------------------------------------ */
static int32_t hk_proper(const int32_t* label, int32_t a) {
    while (label[a] != a) a = label[a];
    return a;
}

static void hk_merge(int32_t* label, int32_t a, int32_t b) {
    a = hk_proper(label, a);
    b = hk_proper(label, b);
    if (a < b) label[b] = a;
    else if (b < a) label[a] = b;
}

void or_label(int L, const uint8_t* bond_r, const uint8_t* bond_d, int32_t* label) {
    int64_t N = (int64_t)L * L;
    /* Raster scan: each site looks back at its left and upper neighbours
     * (the bonds owned by them), without wrapping. */
    for (int y = 0; y < L; ++y) {
        for (int x = 0; x < L; ++x) {
            int32_t i = (int32_t)((int64_t)y * L + x);
            int left = (x > 0) && bond_r[i - 1];
            int up = (y > 0) && bond_d[i - L];
            if (!left && !up) {
                label[i] = i; /* a new cluster starts here */
            } else if (left && !up) {
                label[i] = hk_proper(label, i - 1);
            } else if (!left && up) {
                label[i] = hk_proper(label, i - L);
            } else {
                int32_t a = hk_proper(label, i - 1);
                int32_t b = hk_proper(label, i - L);
                label[i] = (a < b) ? a : b;
                hk_merge(label, a, b);
            }
        }
    }
    /* Periodic boundaries: the bonds that wrap from column L-1 to column 0
     * and from row L-1 to row 0. */
    for (int y = 0; y < L; ++y) {
        int32_t i = (int32_t)((int64_t)y * L + (L - 1));
        if (bond_r[i]) hk_merge(label, i, (int32_t)((int64_t)y * L));
    }
    for (int x = 0; x < L; ++x) {
        int32_t i = (int32_t)((int64_t)(L - 1) * L + x);
        if (bond_d[i]) hk_merge(label, i, x);
    }
    /* Every site takes the proper label of its cluster. */
    for (int64_t i = 0; i < N; ++i) label[i] = hk_proper(label, (int32_t)i);
}

/* ------------------------------------------------------------------ */
/* Step 3: spin flip, Sec. 2 steps (v)-(vii) (R6).                          */
/* ------------------------------------------------------------------ */
/* R6: the word W that decides the new value of the cluster with canonical
 * label rho.  Two-outcome cases (Potts q = 2, the clock reflection): the
 * cluster's bit B, given as W = B * 2^31; otherwise word 0 of its draw. */
static uint32_t cluster_word(int q, int model, uint64_t seed, uint32_t rho, uint64_t t) {
    uint32_t w[4];
    if (model == OR_CLOCK || q == 2) {
        or_draw(seed, rho >> 7, t, OR_P_CLUSTER, w);
        const uint32_t bit = (w[(rho & 127u) >> 5] >> (rho & 31u)) & 1u;
        return bit << 31;
    }
    or_draw(seed, rho, t, OR_P_CLUSTER, w);
    return w[0];
}

/* New value of a site with old value s in a cluster whose draw is W. */
static int8_t flip_value(int q, int model, int m, uint32_t W, int8_t s) {
    if (model == OR_POTTS) return (int8_t)or_qmap(W, (uint32_t)q);
    if (W >= 0x80000000u) return (int8_t)(((m - s) % q + q) % q);
    return s;
}

void or_flip(int L, int q, int model, uint64_t seed, uint64_t t, const int32_t* label,
             int8_t* spins) {
    int64_t N = (int64_t)L * L;
    int m = (model == OR_CLOCK) ? or_mirror(q, seed, t) : 0;
    /* One draw per cluster, made at the cluster's proper label. */
    uint32_t* cluster_word_of = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)N);
    for (int64_t i = 0; i < N; ++i) {
        if (label[i] == i) cluster_word_of[i] = cluster_word(q, model, seed, (uint32_t)i, t);
    }
    for (int64_t i = 0; i < N; ++i) spins[i] = flip_value(q, model, m, cluster_word_of[label[i]], spins[i]);
    free(cluster_word_of);
}

void or_flip_at(int q, int model, uint64_t seed, uint64_t t, int64_t n, const int32_t* root,
                const int8_t* old, int8_t* out) {
    int m = (model == OR_CLOCK) ? or_mirror(q, seed, t) : 0;
    for (int64_t k = 0; k < n; ++k)
        out[k] = flip_value(q, model, m, cluster_word(q, model, seed, (uint32_t)root[k], t), old[k]);
}

int64_t or_sweep(int L, int q, int model, const uint32_t* table, uint64_t seed, uint64_t t,
                 int8_t* spins, uint8_t* bond_r, uint8_t* bond_d, int32_t* label) {
    int64_t N = (int64_t)L * L;
    or_bonds(L, q, model, table, seed, t, spins, bond_r, bond_d);
    or_label(L, bond_r, bond_d, label);
    or_flip(L, q, model, seed, t, label, spins);
    int64_t clusters = 0;
    for (int64_t i = 0; i < N; ++i) clusters += (label[i] == i);
    return clusters;
}

/* ------------------------------------------------------------------ */
/* Measurements (Sec. 4).                                                   */
/* ------------------------------------------------------------------ */
void or_counts(int L, int q, const int8_t* spins, int64_t* hist, int64_t* pair_hist) {
    for (int k = 0; k < q; ++k) hist[k] = 0, pair_hist[k] = 0;
    for (int y = 0; y < L; ++y) {
        for (int x = 0; x < L; ++x) {
            int s = spins[(int64_t)y * L + x];
            int sr = spins[(int64_t)y * L + (x + 1) % L];
            int sd = spins[(int64_t)((y + 1) % L) * L + x];
            hist[s] += 1;
            pair_hist[((sr - s) % q + q) % q] += 1;
            pair_hist[((sd - s) % q + q) % q] += 1;
        }
    }
}

/* Correlation counts at distance r (Sec. 4, the clock model's correlation
 * function): over every site i and both lattice directions, the histogram of
 * (s_j - s_i) mod q for the site j = i + r in that direction (periodic).
 * 2N pairs in all. */
void or_corr_counts(int L, int q, const int8_t* spins, int r, int64_t* corr_hist) {
    for (int k = 0; k < q; ++k) corr_hist[k] = 0;
    for (int y = 0; y < L; ++y) {
        for (int x = 0; x < L; ++x) {
            int s = spins[(int64_t)y * L + x];
            int sx = spins[(int64_t)y * L + (x + r) % L];
            int sy = spins[(int64_t)((y + r) % L) * L + x];
            corr_hist[((sx - s) % q + q) % q] += 1;
            corr_hist[((sy - s) % q + q) % q] += 1;
        }
    }
}

/* G(r) = <S_i^x S_{i+r}^x + S_i^y S_{i+r}^y>: the mean over the 2N pairs of
 * cos(theta_j - theta_i), theta = 2 pi s / q, from the counts above. */
double or_corr_g(int L, int q, const int64_t* corr_hist) {
    double N = (double)L * (double)L;
    double g = 0.0;
    for (int d = 0; d < q; ++d) g += (double)corr_hist[d] * cos_turn(d, q);
    return g / (2.0 * N);
}

void or_observables(int L, int q, int model, double J, const int64_t* hist,
                    const int64_t* pair_hist, double* e_per_site, double* m2) {
    double N = (double)L * (double)L;
    if (model == OR_POTTS) {
        /* H = -J sum (delta - 1) = J * (number of unequal neighbour pairs). */
        double unequal = 2.0 * N - (double)pair_hist[0];
        *e_per_site = J * unequal / N;
        /* M^2 = (q sum_k n[k]^2 - N^2) / (q - 1), normalised by N^2. */
        double s2 = 0.0;
        for (int k = 0; k < q; ++k) s2 += (double)hist[k] * (double)hist[k];
        *m2 = ((double)q * s2 - N * N) / ((double)(q - 1) * N * N);
    } else {
        /* H = -J sum S_i . S_j = -J sum_pairs cos(theta_j - theta_i). */
        double e = 0.0;
        for (int d = 0; d < q; ++d) e += (double)pair_hist[d] * cos_turn(d, q);
        *e_per_site = -J * e / N;
        double mx = 0.0, my = 0.0;
        for (int k = 0; k < q; ++k) {
            mx += (double)hist[k] * cos_turn(k, q);
            my += (double)hist[k] * sin_turn(k, q);
        }
        *m2 = (mx * mx + my * my) / (N * N);
    }
}

int or_run(int L, int q, int model, double T, double J, uint64_t seed, int64_t n_therm,
           int64_t n_meas, int8_t* spins, double* e, double* m2) {
    if (!params_ok(L, q, model) || n_therm < 0 || n_meas < 0) return -1;
    int64_t N = (int64_t)L * L;
    uint32_t* table = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)or_table_size(model, q));
    if (or_cutoffs(model, q, T, J, table) < 0) {
        free(table);
        return -1;
    }
    uint8_t* br = (uint8_t*)malloc((size_t)N);
    uint8_t* bd = (uint8_t*)malloc((size_t)N);
    int32_t* lab = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
    or_init(L, q, seed, spins);
    int64_t hist[32], pair[32];
    for (int64_t t = 0; t < n_therm + n_meas; ++t) {
        or_sweep(L, q, model, table, seed, (uint64_t)t, spins, br, bd, lab);
        if (t >= n_therm) {
            or_counts(L, q, spins, hist, pair);
            or_observables(L, q, model, J, hist, pair, &e[t - n_therm], &m2[t - n_therm]);
        }
    }
    free(lab);
    free(bd);
    free(br);
    free(table);
    return 0;
}

int or_transition_counts(int L, int q, int model, double T, double J, const int8_t* s0,
                         uint64_t t, uint64_t seed0, int64_t nseeds, int64_t* counts) {
    if (!params_ok(L, q, model)) return -1;
    int64_t N = (int64_t)L * L;
    double states = pow((double)q, (double)N);
    if (states > 2147483648.0) return -1;
    uint32_t* table = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)or_table_size(model, q));
    if (or_cutoffs(model, q, T, J, table) < 0) {
        free(table);
        return -1;
    }
    int8_t* s = (int8_t*)malloc((size_t)N);
    uint8_t* br = (uint8_t*)malloc((size_t)N);
    uint8_t* bd = (uint8_t*)malloc((size_t)N);
    int32_t* lab = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
    for (int64_t k = 0; k < nseeds; ++k) {
        memcpy(s, s0, (size_t)N);
        or_sweep(L, q, model, table, seed0 + (uint64_t)k, t, s, br, bd, lab);
        int64_t idx = 0;
        for (int64_t i = N - 1; i >= 0; --i) idx = idx * q + s[i];
        counts[idx] += 1;
    }
    free(lab);
    free(bd);
    free(br);
    free(s);
    free(table);
    return 0;
}

/* ------------------------------------------------------------------ */
/* State hashes: SplitMix64 finaliser (Steele, Lea, Flood, OOPSLA 2014).    */
/* ------------------------------------------------------------------ */
uint64_t or_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t or_hash_spins(int64_t n, const int8_t* spins) {
    uint64_t h = 0;
    for (int64_t i = 0; i < n; ++i) h += or_mix64(((uint64_t)i << 8) | (uint8_t)spins[i]);
    return h;
}

uint64_t or_hash_labels(int64_t n, const int32_t* label) {
    uint64_t h = 0;
    for (int64_t i = 0; i < n; ++i) h += or_mix64(((uint64_t)i << 32) | (uint32_t)label[i]);
    return h;
}
