/*
 * ptoracle.c -- plain, single-threaded CPU oracle for parallel-tempering Metropolis
 * sweeps over Suzuki-Trotter replicas of a transverse-field Ising model.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this
 * file: only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * use it.  It shares no code, header, constant or table with the HIP library.
 *
 * What it computes (the paper, Section 2): R Markov chains ("replicas"), each with the
 * stationary distribution of the system at its own rung of a ladder; every chain is
 * swept with single-spin Metropolis flips; after a fixed number of sweeps adjacent
 * chains are swapped with the probability that their states would have at each other's
 * rung; only disjoint neighbouring pairs are candidates, so the swaps of one step are
 * independent (Section 2, "every two neighboring chains").  Each chain is a classical
 * system of M coupled copies of the Ising problem (Section 6, M = 128 in the paper;
 * the Suzuki-Trotter mapping of reference [14]).
 *
 * Readings where the paper is silent (each listed with its reason in the design notes):
 *   action of replica x at rung r:  S_r(x) = b_r * E_cl(x) - K_r * C(x)
 *     E_cl = sum_k [ sum_edges J_ij s_i^k s_j^k + sum_i h_i s_i^k ]
 *     C    = sum_k sum_i s_i^k s_i^{(k+1) mod M}        (C = 0 when M == 1)
 *   sweep order: colour classes (slice parity p, spatial colour g); a class is an
 *     independent set, so the order inside a class cannot change the result;
 *   acceptance: flip iff u <= thr(dS) with u a 32-bit Philox word, thr from
 *     or_metropolis_threshold (acceptance probability (thr+1)/2^32);
 *   swaps: deterministic even/odd pairs (r, r+1), r = e mod 2, at exchange step e;
 *     swaps exchange the rung labels of the replicas, not their spins;
 *   random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), counter
 *     keyed by (site and slice group, sweep, replica slot, instance) -- see or_flip_word.
 *
 * Floating point: FP64 throughout; build with -ffp-contract=off and without
 * -ffast-math so every product and sum is a separately rounded IEEE operation.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Imaginary-time correlation lags accumulated per rung (see or_tau_lag). */
#define OR_TAU_LAGS 8

#define OR_LABEL_NONE 0
#define OR_LABEL_UP 1
#define OR_LABEL_DOWN 2

/* RNG domains: the second key word is xor-ed with one of these. */
#define OR_DOMAIN_FLIP 0x00000000u
#define OR_DOMAIN_SWAP 0x53574150u /* 'SWAP' */
#define OR_DOMAIN_INIT 0x494E4954u /* 'INIT' */

typedef struct {
    int32_t index;  /* instance number n: enters every random counter */
    int32_t N, M, R, n_edges, n_colors;
    const int32_t *edge_i, *edge_j; /* undirected, listed once */
    const int8_t *edge_J;
    const int8_t *h;
    const uint8_t *color;
    const double *b, *K;            /* per rung; rung 0 is the coldest */
} or_instance;

typedef struct {
    int8_t *s;           /* [R][M][N] by replica slot c */
    int32_t *rung_of;    /* [R]  slot -> rung */
    int32_t *replica_of; /* [R]  rung -> slot */
    int64_t *E;          /* [R]  E_cl by slot */
    int64_t *C;          /* [R]  C by slot */
    int8_t *label;       /* [R]  by slot */
    uint64_t *rt;        /* [R]  completed round trips by slot */
    uint64_t *acc;       /* [R-1] accepted swaps of pair (r, r+1) */
    uint64_t *att;       /* [R-1] attempted swaps of pair (r, r+1) */
    int64_t *sumE, *sumC, *sumE2, *sumC2; /* [R] by rung */
    uint64_t *nup, *ndown; /* [R] by rung: exchange steps at which the replica there was
                              labelled UP / DOWN */
    uint64_t *counters;  /* [0] sweeps t, [1] exchange steps e, [2] n_acc */
    int64_t *sumCt;      /* [R][OR_TAU_LAGS] by rung: sum over exchange steps of the
                            replica's Ct_l (or_tau_corr) */
} or_state;

/* ------------------------------------------------------------------ Philox4x32-10 */

/* One Philox4x32 evaluation with ten rounds.  Round function and constants are those
 * published by Salmon et al. (SC'11): two 32x32->64 products with multipliers
 * 0xD2511F53 and 0xCD9E8D57, the high halves xor-ed with the other two words and the
 * round key; the key is bumped by the Weyl increments 0x9E3779B9, 0xBB67AE85. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int round = 0; round < 10; ++round) {
        uint64_t prod_a = (uint64_t)0xD2511F53u * (uint64_t)x[0];
        uint64_t prod_b = (uint64_t)0xCD9E8D57u * (uint64_t)x[2];
        uint32_t y0 = (uint32_t)(prod_b >> 32) ^ x[1] ^ k[0];
        uint32_t y1 = (uint32_t)prod_b;
        uint32_t y2 = (uint32_t)(prod_a >> 32) ^ x[3] ^ k[1];
        uint32_t y3 = (uint32_t)prod_a;
        x[0] = y0; x[1] = y1; x[2] = y2; x[3] = y3;
        k[0] += 0x9E3779B9u;
        k[1] += 0xBB67AE85u;
    }
    out[0] = x[0]; out[1] = x[1]; out[2] = x[2]; out[3] = x[3];
}

static void key_for(uint64_t seed, uint32_t domain, uint32_t key[2])
{
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32) ^ domain;
}

/* Random counters of a spin draw.  Slice k has parity p = k mod 2 and index m = k div 2
 * within its parity (M == 1: p = m = 0).  The four same-parity slices m = 4g..4g+3 of
 * one site share one Philox call, word (m mod 4):
 *   ctr0 = (2 i + p) * ceil(Mh / 4) + m div 4,  Mh = M / 2 (1 when M == 1). */
static int32_t slice_groups(int32_t M) { int32_t Mh = (M >= 2) ? M / 2 : 1; return (Mh + 3) / 4; }

static uint32_t spin_counter0(int32_t M, int32_t k, int32_t i)
{
    int32_t p = (M >= 2) ? (k & 1) : 0;
    int32_t m = (M >= 2) ? (k >> 1) : 0;
    return ((uint32_t)(2 * i + p)) * (uint32_t)slice_groups(M) + (uint32_t)(m >> 2);
}

static int32_t spin_word(int32_t M, int32_t k)
{
    int32_t m = (M >= 2) ? (k >> 1) : 0;
    return m & 3;
}

/* Word used by the flip attempt of (instance n, slot c, sweep t, slice k, site i):
 * word (m mod 4) of Philox(ctr = (spin_counter0, t, c, n)). */
uint32_t or_flip_word(uint64_t seed, int32_t n, int32_t M, int32_t c, uint64_t t,
                      int32_t k, int32_t i)
{
    uint32_t key[2], ctr[4], out[4];
    key_for(seed, OR_DOMAIN_FLIP, key);
    ctr[0] = spin_counter0(M, k, i);
    ctr[1] = (uint32_t)t;
    ctr[2] = (uint32_t)c;
    ctr[3] = (uint32_t)n;
    or_philox4x32_10(ctr, key, out);
    return out[spin_word(M, k)];
}

/* Word used by the swap attempt of pair (r, r+1) at exchange step e:
 * word 0 of Philox(ctr = (r, e, 0, n)) in the SWAP domain. */
uint32_t or_swap_word(uint64_t seed, int32_t n, int32_t r, uint64_t e)
{
    uint32_t key[2], ctr[4], out[4];
    key_for(seed, OR_DOMAIN_SWAP, key);
    ctr[0] = (uint32_t)r;
    ctr[1] = (uint32_t)e;
    ctr[2] = 0u;
    ctr[3] = (uint32_t)n;
    or_philox4x32_10(ctr, key, out);
    return out[0];
}

/* Initial spin of (instance n, slot c, slice k, site i): the top bit of word (m mod 4) of
 * Philox(ctr = (spin_counter0, 0, c, n)) in the INIT domain; 1 -> +1. */
int8_t or_init_spin(uint64_t seed, int32_t n, int32_t M, int32_t c, int32_t k, int32_t i)
{
    uint32_t key[2], ctr[4], out[4];
    key_for(seed, OR_DOMAIN_INIT, key);
    ctr[0] = spin_counter0(M, k, i);
    ctr[1] = 0u;
    ctr[2] = (uint32_t)c;
    ctr[3] = (uint32_t)n;
    or_philox4x32_10(ctr, key, out);
    return (out[spin_word(M, k)] >> 31) ? (int8_t)1 : (int8_t)-1;
}

/* ------------------------------------------------------------- deterministic exp */

/* exp(x) for x <= 0 built from IEEE +, -, *, floor and ldexp only, so that any two
 * correct implementations of the same steps agree to the last bit:
 *   n = floor(x*log2(e) + 1/2),  r = (x - n*c1) - n*c2  with c1 + c2 = ln 2,
 *   exp(r) by the degree-12 Taylor polynomial in Horner form, result * 2^n.
 * c1 keeps 32 significant bits of ln 2 (round-down of ln2 * 2^32, divided by 2^32) so
 * n*c1 is exact for |n| < 2^21; c2 is ln2 - c1 rounded to double.  Below -32 the
 * result is returned as 0: exp(-32) * 2^32 < 1, so no threshold can depend on it. */
double or_exp_det(double x)
{
    static const double log2e = 0x1.71547652b82fep+0;          /* 1/ln 2 */
    static const double c1 = 2977044471.0 / 4294967296.0;       /* ln2 high part */
    static const double c2 = 0x1.a39ef35793c76p-33;             /* ln2 - c1 */
    /* 1/j! for j = 0..12, each correctly rounded to double */
    static const double inv_fact[13] = {
        1.0,
        1.0,
        0.5,
        0x1.5555555555555p-3,   /* 1/6 */
        0x1.5555555555555p-5,   /* 1/24 */
        0x1.1111111111111p-7,   /* 1/120 */
        0x1.6c16c16c16c17p-10,  /* 1/720 */
        0x1.a01a01a01a01ap-13,  /* 1/5040 */
        0x1.a01a01a01a01ap-16,  /* 1/40320 */
        0x1.71de3a556c734p-19,  /* 1/362880 */
        0x1.27e4fb7789f5cp-22,  /* 1/3628800 */
        0x1.ae64567f544e4p-26,  /* 1/39916800 */
        0x1.1eed8eff8d898p-29,  /* 1/479001600 */
    };
    if (!(x >= -32.0)) return 0.0;
    double n = floor(x * log2e + 0.5);
    double r = (x - n * c1) - n * c2;
    double p = inv_fact[12];
    for (int j = 11; j >= 0; --j) {
        p = p * r;
        p = p + inv_fact[j];
    }
    return ldexp(p, (int)n);
}

/* Acceptance threshold for an action change dS under the Metropolis rule
 * min(1, exp(-dS)) quantised to 32 bits: a proposal is accepted iff u <= thr for a
 * uniform 32-bit word u, i.e. with probability exactly (thr+1)/2^32.
 *   dS <= 0      -> thr = 2^32 - 1 (always accepted)
 *   dS >  0      -> thr = clamp(floor(exp(-dS) * 2^32), 1, 2^32-1) - 1           */
uint32_t or_metropolis_threshold(double dS)
{
    if (dS <= 0.0) return 0xFFFFFFFFu;
    double v = floor(ldexp(or_exp_det(-dS), 32));
    if (v > 4294967295.0) v = 4294967295.0;
    if (v < 1.0) v = 1.0;
    return (uint32_t)v - 1u;
}

/* --------------------------------------------------------------- adjacency lists */

typedef struct {
    int32_t *start; /* [N+1] */
    int32_t *nbr;   /* [2E] */
    int32_t *J;     /* [2E] */
} or_adj;

static int build_adj(const or_instance *in, or_adj *a)
{
    int32_t N = in->N, E = in->n_edges;
    a->start = (int32_t *)calloc((size_t)N + 1, sizeof(int32_t));
    a->nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * E + 1));
    a->J = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * E + 1));
    int32_t *fill = (int32_t *)calloc((size_t)N + 1, sizeof(int32_t));
    if (!a->start || !a->nbr || !a->J || !fill) { free(fill); return -1; }
    for (int32_t e = 0; e < E; ++e) {
        a->start[in->edge_i[e] + 1]++;
        a->start[in->edge_j[e] + 1]++;
    }
    for (int32_t i = 0; i < N; ++i) a->start[i + 1] += a->start[i];
    for (int32_t e = 0; e < E; ++e) {
        int32_t i = in->edge_i[e], j = in->edge_j[e];
        a->nbr[a->start[i] + fill[i]] = j; a->J[a->start[i] + fill[i]] = in->edge_J[e]; fill[i]++;
        a->nbr[a->start[j] + fill[j]] = i; a->J[a->start[j] + fill[j]] = in->edge_J[e]; fill[j]++;
    }
    free(fill);
    return 0;
}

static void free_adj(or_adj *a) { free(a->start); free(a->nbr); free(a->J); }

static inline int8_t spin_at(const or_instance *in, const int8_t *s, int32_t c, int32_t k,
                             int32_t i)
{
    return s[((size_t)c * in->M + (size_t)k) * in->N + i];
}

/* ------------------------------------------------------------------ energies */

/* E_cl and C of every replica slot, from scratch (definitions in the file header). */
void or_energies(const or_instance *in, const int8_t *s, int64_t *E, int64_t *C)
{
    int32_t N = in->N, M = in->M;
    for (int32_t c = 0; c < in->R; ++c) {
        int64_t e_sum = 0, c_sum = 0;
        for (int32_t k = 0; k < M; ++k) {
            for (int32_t e = 0; e < in->n_edges; ++e)
                e_sum += (int64_t)in->edge_J[e] * spin_at(in, s, c, k, in->edge_i[e]) *
                         spin_at(in, s, c, k, in->edge_j[e]);
            for (int32_t i = 0; i < N; ++i) e_sum += (int64_t)in->h[i] * spin_at(in, s, c, k, i);
            if (M >= 2)
                for (int32_t i = 0; i < N; ++i)
                    c_sum += (int64_t)spin_at(in, s, c, k, i) * spin_at(in, s, c, (k + 1) % M, i);
        }
        E[c] = e_sum;
        C[c] = c_sum;
    }
}

/* ------------------------------------------------------------------ imaginary time */

/* Lag l (0 <= l < OR_TAU_LAGS) of the imaginary-time correlations, in slices:
 * max(1, floor((l + 1) M / 16)), i.e. 1/16 .. 1/2 of the Trotter direction in eighths. */
int32_t or_tau_lag(int32_t M, int32_t l)
{
    int32_t d = (l + 1) * M / 16;
    return d < 1 ? 1 : d;
}

/* Ct_l = sum_k sum_i s_i^k s_i^{(k + lag_l) mod M} of one replica s[M][N]: the spin
 * autocorrelation along the Trotter direction.  Divided by N M it estimates
 * (1/N) sum_i <sigma^z_i(tau) sigma^z_i(0)> at imaginary time tau = lag * beta / M, the
 * correlation whose decay gives the gap above the ground state (the quantity the
 * paper's application, AQUA, computes; Section 1 and its reference [14]). */
void or_tau_corr(const or_instance *in, const int8_t *s, int64_t *out)
{
    int32_t N = in->N, M = in->M;
    for (int32_t l = 0; l < OR_TAU_LAGS; ++l) {
        int32_t lag = or_tau_lag(M, l);
        int64_t acc = 0;
        for (int32_t k = 0; k < M; ++k) {
            int32_t k2 = (k + lag) % M;
            for (int32_t i = 0; i < N; ++i)
                acc += (int64_t)s[(size_t)k * N + i] * s[(size_t)k2 * N + i];
        }
        out[l] = acc;
    }
}

/* ------------------------------------------------------------------ init */

void or_init(const or_instance *in, or_state *st, uint64_t seed)
{
    int32_t N = in->N, M = in->M, R = in->R;
    for (int32_t c = 0; c < R; ++c)
        for (int32_t k = 0; k < M; ++k)
            for (int32_t i = 0; i < N; ++i)
                st->s[((size_t)c * M + k) * N + i] = or_init_spin(seed, in->index, M, c, k, i);
    for (int32_t r = 0; r < R; ++r) {
        st->replica_of[r] = r;
        st->rung_of[r] = r;
        st->label[r] = (r == 0) ? OR_LABEL_UP : OR_LABEL_NONE;
        st->rt[r] = 0;
        st->sumE[r] = st->sumC[r] = st->sumE2[r] = st->sumC2[r] = 0;
        st->nup[r] = st->ndown[r] = 0;
        for (int32_t l = 0; l < OR_TAU_LAGS; ++l) st->sumCt[(size_t)r * OR_TAU_LAGS + l] = 0;
    }
    for (int32_t r = 0; r + 1 < R; ++r) st->acc[r] = st->att[r] = 0;
    st->counters[0] = st->counters[1] = st->counters[2] = 0;
    or_energies(in, st->s, st->E, st->C);
}

/* ------------------------------------------------------------------ sweep */

/* Optional within-class visiting order: when shuffle_seed != 0 the sites of each class
 * are visited in a pseudo-random order (for the order-independence test); the chain
 * itself does not depend on it.  A small xorshift generator, unrelated to Philox. */
static uint64_t xs_next(uint64_t *x)
{
    *x ^= *x << 13; *x ^= *x >> 7; *x ^= *x << 17;
    return *x;
}

/* One single-spin Metropolis attempt at (slot c, slice k, site i) during sweep t. */
static void attempt_flip(const or_instance *in, const or_adj *adj, or_state *st,
                         uint64_t seed, uint64_t t, int32_t c, int32_t k, int32_t i)
{
    int32_t N = in->N, M = in->M;
    int8_t *row = st->s + ((size_t)c * M + k) * N;
    int32_t s = row[i];
    int32_t f = in->h[i];
    for (int32_t e = adj->start[i]; e < adj->start[i + 1]; ++e) f += adj->J[e] * row[adj->nbr[e]];
    int32_t tp = 0;
    if (M >= 2)
        tp = spin_at(in, st->s, c, (k + M - 1) % M, i) + spin_at(in, st->s, c, (k + 1) % M, i);
    int64_t dE = -2 * (int64_t)s * f;   /* change of E_cl if s -> -s */
    int64_t dC = -2 * (int64_t)s * tp;  /* change of C    if s -> -s */
    int32_t rung = st->rung_of[c];
    double b = in->b[rung];
    double K = (M >= 2) ? in->K[rung] : 0.0;
    double dS = b * (double)dE - K * (double)dC;
    uint32_t thr = or_metropolis_threshold(dS);
    uint32_t u = or_flip_word(seed, in->index, M, c, t, k, i);
    if (u <= thr) {
        row[i] = (int8_t)(-s);
        st->E[c] += dE;
        st->C[c] += dC;
    }
}

int or_sweep_ordered(const or_instance *in, or_state *st, uint64_t seed, int32_t n_sweeps,
                     uint64_t shuffle_seed)
{
    or_adj adj;
    if (build_adj(in, &adj)) return -1;
    int32_t N = in->N, M = in->M, R = in->R;
    int32_t P = (M >= 2) ? 2 : 1;
    int32_t *members = (int32_t *)malloc(sizeof(int32_t) * ((size_t)N * M + 1));
    if (!members) { free_adj(&adj); return -1; }
    uint64_t xs = shuffle_seed ? shuffle_seed : 1;
    for (int32_t sw = 0; sw < n_sweeps; ++sw) {
        uint64_t t = st->counters[0];
        for (int32_t p = 0; p < P; ++p) {
            for (int32_t g = 0; g < in->n_colors; ++g) {
                /* the class: every (k, i) with k = p mod 2 and color[i] == g */
                int32_t cnt = 0;
                for (int32_t k = p; k < M; k += P)
                    for (int32_t i = 0; i < N; ++i)
                        if (in->color[i] == g) members[cnt++] = k * N + i;
                for (int32_t c = 0; c < R; ++c) {
                    if (shuffle_seed)
                        for (int32_t a = cnt - 1; a > 0; --a) {
                            int32_t b = (int32_t)(xs_next(&xs) % (uint64_t)(a + 1));
                            int32_t tmp = members[a]; members[a] = members[b]; members[b] = tmp;
                        }
                    for (int32_t m = 0; m < cnt; ++m)
                        attempt_flip(in, &adj, st, seed, t, c, members[m] / N, members[m] % N);
                }
            }
        }
        st->counters[0] = t + 1;
    }
    free(members);
    free_adj(&adj);
    return 0;
}

int or_sweep(const or_instance *in, or_state *st, uint64_t seed, int32_t n_sweeps)
{
    return or_sweep_ordered(in, st, seed, n_sweeps, 0);
}

/* ------------------------------------------------------------------ exchange */

/* One replica-exchange step e: pairs (r, r+1) with r = e mod 2, e mod 2 + 2, ...
 * The log acceptance ratio of exchanging the configurations x (at rung r) and y (at
 * rung r+1) is  S_r(x) + S_{r+1}(y) - S_r(y) - S_{r+1}(x)
 *             = (b_r - b_{r+1})(E_x - E_y) - (K_r - K_{r+1})(C_x - C_y) =: D,
 * accepted with probability min(1, exp(D)), i.e. iff u <= threshold(-D). */
void or_exchange(const or_instance *in, or_state *st, uint64_t seed)
{
    int32_t R = in->R, M = in->M;
    uint64_t e = st->counters[1];
    for (int32_t r = (int32_t)(e & 1u); r + 1 < R; r += 2) {
        int32_t x = st->replica_of[r], y = st->replica_of[r + 1];
        double dE = (double)(st->E[x] - st->E[y]);
        double dC = (double)(st->C[x] - st->C[y]);
        double db = in->b[r] - in->b[r + 1];
        double dK = (M >= 2) ? (in->K[r] - in->K[r + 1]) : 0.0;
        double D = db * dE - dK * dC;
        uint32_t thr = or_metropolis_threshold(-D);
        uint32_t u = or_swap_word(seed, in->index, r, e);
        st->att[r] += 1;
        if (u <= thr) {
            st->replica_of[r] = y;
            st->replica_of[r + 1] = x;
            st->rung_of[y] = r;
            st->rung_of[x] = r + 1;
            st->acc[r] += 1;
        }
    }
    /* round-trip labels: a replica reaching the coldest rung after the hottest one
     * completes a round trip; reaching the hottest rung turns UP into DOWN. */
    int32_t cold = st->replica_of[0], hot = st->replica_of[R - 1];
    if (st->label[cold] == OR_LABEL_DOWN) {
        st->rt[cold] += 1;
        st->label[cold] = OR_LABEL_UP;
    } else if (st->label[cold] == OR_LABEL_NONE) {
        st->label[cold] = OR_LABEL_UP;
    }
    if (st->label[hot] == OR_LABEL_UP) st->label[hot] = OR_LABEL_DOWN;
    /* per-rung accumulators, including the label of the replica found at each rung */
    for (int32_t r = 0; r < R; ++r) {
        int32_t c = st->replica_of[r];
        if (st->label[c] == OR_LABEL_UP) st->nup[r] += 1;
        if (st->label[c] == OR_LABEL_DOWN) st->ndown[r] += 1;
        st->sumE[r] += st->E[c];
        st->sumC[r] += st->C[c];
        st->sumE2[r] += st->E[c] * st->E[c];
        st->sumC2[r] += st->C[c] * st->C[c];
        int64_t ct[OR_TAU_LAGS];
        or_tau_corr(in, st->s + (size_t)c * in->M * in->N, ct);
        for (int32_t l = 0; l < OR_TAU_LAGS; ++l) st->sumCt[(size_t)r * OR_TAU_LAGS + l] += ct[l];
    }
    st->counters[2] += 1;
    st->counters[1] = e + 1;
}

/* ------------------------------------------------------------------ cycles */

/* n_cycles x { k sweeps; one exchange step } (the loop of the paper's Figures 4-6). */
int or_run(const or_instance *in, or_state *st, uint64_t seed, int32_t k, int32_t n_cycles)
{
    for (int32_t cyc = 0; cyc < n_cycles; ++cyc) {
        if (or_sweep(in, st, seed, k)) return -1;
        or_exchange(in, st, seed);
    }
    return 0;
}
