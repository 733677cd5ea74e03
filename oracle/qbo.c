/*
 * qbo.c -- CPU oracle for the IC-D^2S hot path (TEST INFRASTRUCTURE ONLY).
 *
 * Plain loops, int64 accumulators, no blocking, no fusion.  Each function
 * names the passage of the paper it follows.  Readings where the paper is
 * silent or inconsistent are marked "Reading:".  Build with
 *   gcc -O2 -ffp-contract=off -fPIC -shared -o libqbo.so qbo.c -lm
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg use
 * this file.  It shares no code with the GPU library.
 */
#include "qbo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, as published by Salmon et al. (SC'11): a 4-word counter is
 * scrambled by ten rounds; each round multiplies words 0 and 2 by fixed odd
 * constants, keeps both halves of the 64-bit products, and mixes the high
 * halves with words 1/3 and the round key.  The key advances by two Weyl
 * constants between rounds.  Pinned by the published known-answer vectors. */
void qbo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static uint32_t philox_word(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                            uint64_t seed, int word)
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t out[4];
    qbo_philox4x32_10(ctr, key, out);
    return out[word];
}

/* ------------------------------------------------------------------------ */
/* eq. 1: f(x) = sum_i Q_ii x_i + sum_i sum_{j != i} Q_ij x_i x_j.
 * Pinned: brute force and closed forms in the tests. */
int64_t qbo_energy_def(int n, const int16_t *Q, const uint8_t *x)
{
    int64_t f = 0;
    for (int i = 0; i < n; ++i)
        if (x[i]) f += Q[(int64_t)i * n + i];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (j != i && x[i] && x[j]) f += Q[(int64_t)i * n + j];
    return f;
}

/* Local field h = Q x for every solution (the quantity the 1-flip move
 * values of the Tabu section are built from). */
void qbo_field(int n, const int16_t *Q, int z, const uint8_t *X, int32_t *H)
{
    for (int p = 0; p < z; ++p)
        for (int i = 0; i < n; ++i) {
            int64_t acc = 0;
            for (int j = 0; j < n; ++j)
                acc += (int64_t)Q[(int64_t)i * n + j] * X[(int64_t)p * n + j];
            H[(int64_t)p * n + i] = (int32_t)acc;
        }
}

/* x^T Q x = sum_i x_i (Q x)_i. */
void qbo_energy(int n, int z, const uint8_t *X, const int32_t *H, int64_t *E)
{
    for (int p = 0; p < z; ++p) {
        int64_t acc = 0;
        for (int i = 0; i < n; ++i)
            acc += (int64_t)X[(int64_t)p * n + i] * H[(int64_t)p * n + i];
        E[p] = acc;
    }
}

/* Energy change of flipping x_i:  (1 - 2x_i)(Q_ii + 2 sum_{j != i} Q_ij x_j),
 * written with h = Qx as Q_ii + 2(1 - 2x_i) h_i.
 * Reading: the Tabu listing's move value omits the factor 2 that eq. 4 has;
 * the factor 2 is what makes it equal the exact energy difference. */
int32_t qbo_flip_delta(int n, const int16_t *Q, const uint8_t *x, const int32_t *h, int i)
{
    int32_t qii = Q[(int64_t)i * n + i];
    return qii + 2 * (1 - 2 * (int32_t)x[i]) * h[i];
}

/* Weight_Effect_Extraction: eta_j = sum_i |Q_ij|. */
void qbo_eta(int n, const int16_t *Q, int64_t *eta)
{
    for (int j = 0; j < n; ++j) {
        int64_t acc = 0;
        for (int i = 0; i < n; ++i) {
            int32_t v = Q[(int64_t)i * n + j];
            acc += v < 0 ? -v : v;
        }
        eta[j] = acc;
    }
}

/* Scale of the annealer's temperature schedule and of the learned
 * selector's field features (Reading 14: the IM's temperature is stated in
 * units of the typical local-field size).  sigma = sqrt(S / n) with
 * S = sum over i != j of Q_ij^2, summed exactly in 64-bit integers: the
 * root-mean-square, over the variables, of the field's spread. */
double qbo_sigma(int n, const int16_t *Q)
{
    uint64_t acc = 0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            if (i == j) continue;
            int64_t v = Q[(int64_t)i * n + j];
            acc += (uint64_t)(v * v);
        }
    return sqrt((double)acc / (double)n);
}

/* The same sum over the stored entries of compressed sparse rows (row i's
 * entries col[rowptr[i] .. rowptr[i+1]), values val), skipping the diagonal. */
double qbo_sigma_csr(int n, const int32_t *rowptr, const int32_t *col, const int16_t *val)
{
    uint64_t acc = 0;
    for (int i = 0; i < n; ++i)
        for (int32_t t = rowptr[i]; t < rowptr[i + 1]; ++t) {
            if (col[t] == i) continue;
            int64_t v = val[t];
            acc += (uint64_t)(v * v);
        }
    return sqrt((double)acc / (double)n);
}

/* Generate_Initial_Solution_Set (Alg. 2): z uniformly random binary rows.
 * Reading: bit = top bit of a Philox word, counter (j/4, p, 0, 3<<28),
 * word j mod 4, key = 64-bit seed. */
void qbo_init_x(int n, int z, uint64_t seed, uint8_t *X)
{
    for (int p = 0; p < z; ++p)
        for (int j = 0; j < n; ++j) {
            uint32_t u = philox_word((uint32_t)(j >> 2), (uint32_t)p, 0u, 3u << 28, seed, j & 3);
            X[(int64_t)p * n + j] = (uint8_t)(u >> 31);
        }
}

/* ------------------------------------------------------------------------ */
/* Tabu search, Alg. 1, with the readings:
 *  - move value = exact energy difference (factor 2, flip direction);
 *  - OV adds the move value of the chosen variable taken before the flip;
 *  - a tabu move is still allowed when it would reach a new best objective
 *    (aspiration, stated in the text of the Tabu section; flag-selectable);
 *  - argmin ties go to the lowest index; if every variable is tabu and none
 *    aspirates, the argmin is taken over all variables;
 *  - tenure vector C starts at 0 on every call; C_i += c, then every positive
 *    entry is decremented (so a flipped variable is blocked c-1 steps);
 *  - the call returns x_min (the best seen) and its field; T counts flips.
 * Parity status: pinned by the hand-worked fixture in tests/golden, by the
 * incremental-vs-recomputed field and energy invariants, by reaching the
 * brute-force optimum on tiny instances, and by move-by-move replays of
 * whole runs against move values brute-forced from eq. 1. */
void qbo_tabu(int n, const int16_t *Q, uint8_t *x, int32_t *h, int64_t *ov,
              int alpha, int tenure, int aspiration, int32_t *T, int32_t *lastflip)
{
    int32_t *C = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    uint8_t *xmin = (uint8_t *)malloc((size_t)n);
    memcpy(xmin, x, (size_t)n);
    for (int j = 0; j < n; ++j) { T[j] = 0; lastflip[j] = 0; }
    int64_t OV = *ov, OVmin = OV;

    for (int step = 1; step <= alpha; ++step) {
        int best = -1;
        int32_t bestd = 0;
        for (int k = 0; k < n; ++k) {
            int32_t d = qbo_flip_delta(n, Q, x, h, k);
            int allowed = C[k] <= 0 || (aspiration && OV + d < OVmin);
            if (allowed && (best < 0 || d < bestd)) { best = k; bestd = d; }
        }
        if (best < 0) {
            for (int k = 0; k < n; ++k) {
                int32_t d = qbo_flip_delta(n, Q, x, h, k);
                if (best < 0 || d < bestd) { best = k; bestd = d; }
            }
        }
        int i = best;
        OV += bestd;
        int32_t s = 1 - 2 * (int32_t)x[i];
        for (int j = 0; j < n; ++j) h[j] += s * Q[(int64_t)j * n + i];
        x[i] ^= 1;
        T[i] += 1;
        lastflip[i] = step;
        C[i] += tenure;
        for (int j = 0; j < n; ++j)
            if (C[j] > 0) C[j] -= 1;
        if (OV < OVmin) {
            OVmin = OV;
            memcpy(xmin, x, (size_t)n);
        }
    }
    /* return x_min: move the field to x_min by undoing the differing bits */
    for (int j = 0; j < n; ++j)
        if (x[j] != xmin[j]) {
            int32_t s = (int32_t)xmin[j] - (int32_t)x[j];
            for (int i = 0; i < n; ++i) h[i] += s * Q[(int64_t)i * n + j];
            x[j] = xmin[j];
        }
    *ov = OVmin;
    free(C);
    free(xmin);
}

/* ------------------------------------------------------------------------ */
/* Control parameters and their aggregation (Alg. 4):
 *   eta_hat_j = eta_j / eta_max                    (Reading: normalised)
 *   gamma_j   = 1 - |sum_p X_pj - z/2| / (z/2)      = (z - |2 c_j - z|) / z
 *   Delta_pj  = 1 - T_pj / max_j T_pj               (Reading: max T := 1 if 0)
 *   A_pj      = w1 eta_hat_j + w2 gamma_j - w3 Delta_pj
 * K_pj = A_pj * (eta_max * z * T'_p) * Wd, an exact integer with the same
 * order as A_pj within each solution.  Pinned in the tests against exact
 * rational arithmetic. */
void qbo_keys(int n, int z, const int64_t *eta, const uint8_t *X, const int32_t *T,
              int W1, int W2, int W3, int64_t *K)
{
    int64_t eta_max = 1;
    for (int j = 0; j < n; ++j)
        if (eta[j] > eta_max) eta_max = eta[j];
    for (int p = 0; p < z; ++p) {
        int64_t Tp = 1;
        for (int j = 0; j < n; ++j)
            if (T[(int64_t)p * n + j] > Tp) Tp = T[(int64_t)p * n + j];
        for (int j = 0; j < n; ++j) {
            int64_t cnt = 0;
            for (int q = 0; q < z; ++q) cnt += X[(int64_t)q * n + j];
            int64_t dev = 2 * cnt - z;
            if (dev < 0) dev = -dev;
            int64_t g = (int64_t)z - dev;                  /* gamma_j * z  */
            int64_t dl = Tp - T[(int64_t)p * n + j];       /* Delta_pj * Tp */
            K[(int64_t)p * n + j] = (int64_t)W1 * eta[j] * z * Tp
                                  + (int64_t)W2 * g * eta_max * Tp
                                  - (int64_t)W3 * dl * eta_max * z;
        }
    }
}

static const int64_t *g_sort_keys;
static int cmp_key_desc_index_asc(const void *a, const void *b)
{
    int32_t ia = *(const int32_t *)a, ib = *(const int32_t *)b;
    int64_t ka = g_sort_keys[ia], kb = g_sort_keys[ib];
    if (ka != kb) return ka > kb ? -1 : 1;
    return ia < ib ? -1 : (ia > ib);
}

/* Rank order of Alg. 3 ("variables with the highest values in A").
 * Reading: ties go to the lower index. */
void qbo_order(int n, const int64_t *K, int32_t *order)
{
    for (int j = 0; j < n; ++j) order[j] = j;
    g_sort_keys = K;
    qsort(order, (size_t)n, sizeof(int32_t), cmp_key_desc_index_asc);
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return x < y ? -1 : (x > y);
}

/* ------------------------------------------------------------------------ */
/* Sub-QUBO of eq. 4 for the variables S of one solution:
 *   b_i = sum_{j not in S} 2 Q_ij x_j,  linear term c_i = Q_ii + b_i,
 *   quadratic part Q_ij for i != j in S (Reading: the diagonal lives only in
 *   the linear term, Alg. 3 adds b to the diagonal of Q').
 * F0_a = c_a + 2 sum_{b != a} T_ab y0_b is the flip basis of the annealer:
 * flipping y_a changes f_S by (1 - 2 y_a) F_a.  Pinned: for every y,
 * f(x with x_S := y) - f_S(y) is the same constant (tests, small m). */
void qbo_extract(int n, const int16_t *Q, const uint8_t *x, const int32_t *h,
                 int m, const int32_t *S, int32_t *Tq, int32_t *c, int32_t *F0, uint8_t *y0)
{
    (void)h;
    uint8_t *inS = (uint8_t *)calloc((size_t)n, 1);
    for (int a = 0; a < m; ++a) inS[S[a]] = 1;
    for (int a = 0; a < m; ++a) {
        int i = S[a];
        int64_t b = 0;
        for (int j = 0; j < n; ++j)
            if (!inS[j]) b += 2 * (int64_t)Q[(int64_t)i * n + j] * x[j];
        c[a] = (int32_t)(Q[(int64_t)i * n + i] + b);
        for (int bb = 0; bb < m; ++bb)
            Tq[(int64_t)a * m + bb] = (a == bb) ? 0 : Q[(int64_t)i * n + S[bb]];
        y0[a] = x[i];
    }
    for (int a = 0; a < m; ++a) {
        int64_t acc = c[a];
        for (int bb = 0; bb < m; ++bb)
            if (bb != a) acc += 2 * (int64_t)Tq[(int64_t)a * m + bb] * y0[bb];
        F0[a] = (int32_t)acc;
    }
    free(inS);
}

int64_t qbo_sub_energy(int m, const int32_t *Tq, const int32_t *c, const uint8_t *y)
{
    int64_t f = 0;
    for (int a = 0; a < m; ++a)
        if (y[a]) f += c[a];
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b)
            if (a != b && y[a] && y[b]) f += Tq[(int64_t)a * m + b];
    return f;
}

/* ------------------------------------------------------------------------ */
/* Temperature of sweep s.  Reading: the paper's cosine waveform (the
 * MRAnnealer of the mutation-rate section) used as the IM's temperature
 * schedule, one half period from tmax down to tmin over the nsw sweeps:
 *   T_s = tmin + 0.5 (tmax - tmin)(1 + cos(pi s / (nsw - 1))). */
double qbo_temperature(int s, int nsw, double tmax, double tmin)
{
    if (nsw <= 1) return tmax;
    return tmin + 0.5 * (tmax - tmin) * (1.0 + cos(M_PI * (double)s / (double)(nsw - 1)));
}

/* Metropolis acceptance "u <= exp(-dE/T)" with u quantised to the midpoint of
 * bucket b of 2^B equal buckets, solved for an integer dE:
 *   thr[s][b] = floor(T_s * (-ln((b + 1/2) / 2^B))), capped at 2^31 - 1. */
void qbo_threshold_table(int nsw, int B, double tmax, double tmin, int32_t *thr)
{
    int nb = 1 << B;
    for (int s = 0; s < nsw; ++s) {
        double T = qbo_temperature(s, nsw, tmax, tmin);
        for (int b = 0; b < nb; ++b) {
            double v = T * (-log(((double)b + 0.5) / (double)nb));
            int32_t t = v >= 2147483647.0 ? 2147483647 : (int32_t)floor(v);
            thr[(int64_t)s * nb + b] = t;
        }
    }
}

/* MRAnnealer: r_t = 0.3 (1 + cos(pi t / 15)) 0.99^t (mutation-rate section). */
double qbo_mutation_rate(int t)
{
    return 0.3 * (1.0 + cos(M_PI * (double)t / 15.0)) * pow(0.99, (double)t);
}

/* ------------------------------------------------------------------------ */
/* The Ising-machine stage.  The paper treats the IM as a black box (it was
 * simulated); Reading: a Metropolis annealer in QUBO form, warm-started from
 * the current sub-solution, visiting positions 0..m-1 in order in each sweep,
 * returning the final state of each replica.
 *   uniform for (replica r, sweep s, position k):
 *     Philox4x32-10, counter (((k >> 8) << 6) | (k & 63), s, r, (1<<28) | inst),
 *     key (seed low word, seed high word), word (k >> 6) & 3;
 *   accept iff (1 - 2 y_k) F_k <= thr[s][u >> (32 - B)].
 * Parity status: pinned by closed forms (all-accept / none-accept tables),
 * e == f_S(y) - f_S(y0), 1-flip local optimality under a strict-descent
 * table, the acceptance frequency of a single-variable job, and the
 * Boltzmann distribution of x^T Q x reached by many replicas at a fixed
 * temperature. */
void qbo_anneal(int m, const int32_t *Tq, const int32_t *F0, const uint8_t *y0,
                int nsw, int B, const int32_t *thr, int R, uint64_t seed, uint32_t inst,
                uint8_t *Y, int64_t *e)
{
    qbo_anneal_count(m, Tq, F0, y0, nsw, B, thr, R, seed, inst, Y, e, NULL);
}

/* The same sweep; nacc[r] (optional) receives the number of accepted moves
 * of replica r. */
void qbo_anneal_count(int m, const int32_t *Tq, const int32_t *F0, const uint8_t *y0,
                      int nsw, int B, const int32_t *thr, int R, uint64_t seed, uint32_t inst,
                      uint8_t *Y, int64_t *e, int32_t *nacc)
{
    int32_t *F = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    for (int r = 0; r < R; ++r) {
        uint8_t *y = Y + (int64_t)r * m;
        memcpy(y, y0, (size_t)m);
        memcpy(F, F0, sizeof(int32_t) * (size_t)m);
        int64_t acc = 0;
        int32_t na = 0;
        for (int s = 0; s < nsw; ++s) {
            for (int k = 0; k < m; ++k) {
                int32_t dE = y[k] ? -F[k] : F[k];
                uint32_t cw = (uint32_t)(((k >> 8) << 6) | (k & 63));
                uint32_t u = philox_word(cw, (uint32_t)s, (uint32_t)r, (1u << 28) | inst,
                                         seed, (k >> 6) & 3);
                int32_t t = thr[((int64_t)s << B) + (u >> (32 - B))];
                if (dE <= t) {
                    int32_t d = y[k] ? -1 : 1;
                    y[k] ^= 1;
                    acc += dE;
                    ++na;
                    for (int i = 0; i < m; ++i) F[i] += 2 * d * Tq[(int64_t)i * m + k];
                }
            }
        }
        e[r] = acc;
        if (nacc) nacc[r] = na;
    }
    free(F);
}

/* ------------------------------------------------------------------------ */
/* Ising form (eq. 2 and eq. 3).  With s = 2x - 1, x_i x_j = (1 + s_i + s_j +
 * s_i s_j) / 4, so for symmetric Q
 *   4 f(x) = E'(s) + const4,   E'(s) = -sum_{i != j} J_ij s_i s_j - sum_i h_i s_i,
 *   J_ij = -Q_ij (i != j),  h_i = -2 (Q_ii + sum_{j != i} Q_ij),
 *   const4 = 2 sum_i Q_ii + sum_{i != j} Q_ij,
 * i.e. eq. 2 in units of a quarter (every coefficient an integer).
 * Reading: eq. 2's double sum runs over i != j (s_i^2 = 1 is a constant). */
int64_t qbo_ising_from_qubo(int n, const int16_t *Q, int32_t *J, int64_t *h)
{
    int64_t c4 = 0;
    for (int i = 0; i < n; ++i) {
        int64_t r = Q[(int64_t)i * n + i];
        c4 += 2 * (int64_t)Q[(int64_t)i * n + i];
        for (int j = 0; j < n; ++j) {
            J[(int64_t)i * n + j] = i == j ? 0 : -(int32_t)Q[(int64_t)i * n + j];
            if (j != i) {
                r += Q[(int64_t)i * n + j];
                c4 += Q[(int64_t)i * n + j];
            }
        }
        h[i] = -2 * r;
    }
    return c4;
}

/* E'(s) of eq. 2 (i != j), s_i in {-1, +1}. */
int64_t qbo_ising_energy(int n, const int32_t *J, const int64_t *h, const int8_t *s)
{
    int64_t E = 0;
    for (int i = 0; i < n; ++i) {
        E -= h[i] * s[i];
        for (int j = 0; j < n; ++j)
            if (j != i) E -= (int64_t)J[(int64_t)i * n + j] * s[i] * s[j];
    }
    return E;
}

/* The Ising-machine stage in spin form: R replicas of the sequential
 * Metropolis sweep on E'(s) of eq. 2 (symmetric J, zero diagonal), spins in
 * order, the same uniforms as qbo_anneal (position k, sweep, replica,
 * instance), accept iff the change E'(s with s_k flipped) - E'(s) <= thr'.
 * The change is 2 s_k g_k with the local field g_k = 2 sum_{j != k} J_kj s_j
 * + h_k.  S[R][m] final spins, e[R] = E'(S_r) - E'(s0).  For an Ising form
 * made from a sub-QUBO, thr' = 4 thr gives qbo_anneal's trajectory. */
void qbo_anneal_ising(int m, const int32_t *J, const int64_t *h, const int8_t *s0, int nsw, int B,
                      const int64_t *thr4, int R, uint64_t seed, uint32_t inst, int8_t *S, int64_t *e)
{
    int64_t *g = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    for (int r = 0; r < R; ++r) {
        int8_t *s = S + (int64_t)r * m;
        memcpy(s, s0, (size_t)m);
        for (int k = 0; k < m; ++k) {
            int64_t acc = h[k];
            for (int j = 0; j < m; ++j)
                if (j != k) acc += 2 * (int64_t)J[(int64_t)k * m + j] * s[j];
            g[k] = acc;
        }
        int64_t tot = 0;
        for (int sw = 0; sw < nsw; ++sw) {
            for (int k = 0; k < m; ++k) {
                const int64_t dE = 2 * (int64_t)s[k] * g[k];
                uint32_t cw = (uint32_t)(((k >> 8) << 6) | (k & 63));
                uint32_t u = philox_word(cw, (uint32_t)sw, (uint32_t)r, (1u << 28) | inst, seed, (k >> 6) & 3);
                if (dE <= thr4[((int64_t)sw << B) + (u >> (32 - B))]) {
                    const int sk = s[k];
                    s[k] = (int8_t)-sk;
                    tot += dE;
                    /* g_j changes by 2 J_jk (s_k new - s_k old) = -4 J_jk s_k old */
                    for (int j = 0; j < m; ++j)
                        if (j != k) g[j] -= 4 * (int64_t)J[(int64_t)j * m + k] * sk;
                }
            }
        }
        e[r] = tot;
    }
    free(g);
}

/* ------------------------------------------------------------------------ */
/* Mutation (end of the proposed-heuristic section):
 *   candidates = variables the IM did not solve (not in U);
 *   subset = the floor((n - |U|) * r_t) candidates with the highest A
 *            (Reading: the paper's (n - m) r with m = |U|; ties to lower index);
 *   flip probability = A normalised min-max over all n variables of the
 *     solution (Reading), as the integer threshold
 *     P_j = min(floor(2^32 (K_j - K_lo) / (K_hi - K_lo)), 2^32 - 1)
 *     (P = 2^31 when K_hi == K_lo);
 *   flip iff u_j < P_j with u_j = Philox word j mod 4 of counter
 *     (j/4, t, p, 2<<28). */
int qbo_mutate(int n, uint8_t *x, const int64_t *K, const uint8_t *inU, int t, int p,
               uint64_t seed, uint8_t *flip)
{
    return qbo_mutate2(n, x, K, K, inU, t, p, seed, flip);
}

int qbo_mutate2(int n, uint8_t *x, const int64_t *Korder, const int64_t *Kprob, const uint8_t *inU, int t,
                int p, uint64_t seed, uint8_t *flip)
{
    const int64_t *K = Kprob;
    int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int nc = 0;
    for (int j = 0; j < n; ++j) {
        flip[j] = 0;
        if (!inU[j]) cand[nc++] = j;
    }
    double r = qbo_mutation_rate(t);
    int k = (int)floor((double)nc * r);
    if (k > nc) k = nc;
    g_sort_keys = Korder;
    qsort(cand, (size_t)nc, sizeof(int32_t), cmp_key_desc_index_asc);
    int64_t klo = K[0], khi = K[0];
    for (int j = 1; j < n; ++j) {
        if (K[j] < klo) klo = K[j];
        if (K[j] > khi) khi = K[j];
    }
    for (int a = 0; a < k; ++a) {
        int j = cand[a];
        uint64_t P;
        if (khi == klo) {
            P = 1ull << 31;
        } else {
            unsigned __int128 num = (unsigned __int128)(uint64_t)(K[j] - klo) << 32;
            unsigned __int128 q = num / (unsigned __int128)(uint64_t)(khi - klo);
            P = q > 0xffffffffu ? 0xffffffffull : (uint64_t)q;
        }
        uint32_t u = philox_word((uint32_t)(j >> 2), (uint32_t)t, (uint32_t)p, 2u << 28, seed, j & 3);
        if ((uint64_t)u < P) {
            x[j] ^= 1;
            flip[j] = 1;
        }
    }
    free(cand);
    return k;
}

/* Reading for the ablation without the control parameters (No_SM, the
 * Discussion section): every place where the method ranks variables by A
 * ranks them by a fresh uniform random key instead, one 32-bit Philox word
 * per variable and iteration (stream tag 4), and the mutation flips each of
 * its candidates with probability 1/2. */
void qbo_random_keys(int n, int z, int t, uint64_t seed, int64_t *K)
{
    for (int p = 0; p < z; ++p)
        for (int j = 0; j < n; ++j)
            K[(int64_t)p * n + j] =
                (int64_t)philox_word((uint32_t)(j >> 2), (uint32_t)t, (uint32_t)p, 4u << 28, seed, j & 3);
}

/* ------------------------------------------------------------------------ */
uint16_t qbo_bf16_rne(float f);
void qbo_features(int n, int z, const int16_t *Q, const int64_t *eta, const uint8_t *X, const int32_t *H,
                  const int32_t *T, const int32_t *LF, const int32_t *G, int alpha, const float *sc, uint16_t *F);
void qbo_mlp_scores(int count, const uint16_t *W, const uint16_t *F, float *score, int64_t *K);

static void best_update(int n, int z, const uint8_t *X, const int64_t *E,
                        uint8_t *xbest, int64_t *ebest)
{
    for (int p = 0; p < z; ++p)
        if (E[p] < *ebest) {
            *ebest = E[p];
            memcpy(xbest, X + (int64_t)p * n, (size_t)n);
        }
}

/* Write-back (the last step of Alg. 3): the replica with the lowest e (lowest r on
 * ties) replaces x_S -- unconditionally as in the listing, or, in the
 * "only if not worse" variant, only when its e <= 0.  Returns 1 if written. */
static int pick_and_write(int m, const int32_t *S, const uint8_t *Y, const int64_t *e, int R,
                          int not_worse, uint8_t *x)
{
    int rb = 0;
    for (int r = 1; r < R; ++r)
        if (e[r] < e[rb]) rb = r;
    if (not_worse && e[rb] > 0) return 0;
    for (int a = 0; a < m; ++a) x[S[a]] = Y[(int64_t)rb * m + a];
    return 1;
}

/* Alg. 2 with Call_IM_Solution_Set and Call_IM_Partial_Solution_Set (Alg. 3):
 *   X <- random set; h, E; best.
 *   Initial pass (Reading): contiguous blocks [l m0, (l+1) m0), l < floor(n/m0),
 *     solved one block after another (each block sees the bias of the
 *     previous blocks' results), one job per solution per block.
 *   For t = 0 .. iters-1:
 *     Tabu on every solution; best.
 *     keys K from (eta, Delta from T, gamma from X); per solution the top
 *       sum_q m_pq ranks, job q taking ranks [sum_{<q} m, sum_{<=q} m),
 *       each job's indices ascending (Reading for several IMs per solution).
 *     All jobs extracted against the state before the launch, annealed
 *       (instance number = running job count), best replica (lowest e, lowest
 *       replica on ties) written back unconditionally; h, E; best.
 *     Mutation with r_t; h, E; best.
 *   Best: strictly lower energy wins, scanning solutions in order, so ties go
 *   to the earliest stage and the lowest solution index.
 *   Learned selection (cfg->mlp_W != NULL): the IM variables are the top
 *   MLP scores of the eight features instead of the top A; mutation still
 *   uses A.  G (gain of the last IM job that changed a variable) feeds
 *   feature 4.
 *   Variants: random_select (No_SM: random keys rank the IM variables and
 *   order the mutation candidates, each flipped with probability 1/2);
 *   no_im (No_IM: no sub-QUBOs, so every variable is a mutation candidate);
 *   init_jacobi (all initial blocks of a solution extracted against the
 *   same state and written back together, the concurrent option of the
 *   initial pass); wb_not_worse (a sub-solution is written back only if its
 *   e <= 0); patience (stall termination: stop once E_best has not improved
 *   for that many consecutive iterations). */
int qbo_run(const int16_t *Q, const qbo_run_cfg *cfg, uint8_t *X, int32_t *H, int64_t *E,
            uint8_t *xbest, int64_t *ebest, int64_t *trace_best)
{
    const int n = cfg->n, z = cfg->z, kj = cfg->jobs_per_sol;
    for (int p = 0; p < z; ++p) {
        int64_t tot = 0;
        for (int q = 0; q < kj; ++q) {
            if (cfg->job_m[p * kj + q] < 1) return -1;
            tot += cfg->job_m[p * kj + q];
        }
        if (tot > n) return -1;
    }
    const int learned = cfg->mlp_W != NULL;
    if (learned && (cfg->random_select || cfg->no_im || cfg->wb_not_worse)) return -1;
    int64_t *eta = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *K0 = (int64_t *)calloc((size_t)n * z, sizeof(int64_t));
    int64_t *KR = (int64_t *)malloc(sizeof(int64_t) * (size_t)n * z);
    int32_t *T = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * z);
    int32_t *LF = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * z);
    int32_t *G = (int32_t *)calloc((size_t)n * z, sizeof(int32_t));
    int64_t *K = (int64_t *)malloc(sizeof(int64_t) * (size_t)n * z);
    int64_t *KL = (int64_t *)malloc(sizeof(int64_t) * (size_t)n * z);
    uint16_t *F = (uint16_t *)malloc(sizeof(uint16_t) * 8 * (size_t)n * z);
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    uint8_t *X0 = (uint8_t *)malloc((size_t)n * z);
    int mmax = cfg->init_m;
    for (int i = 0; i < z * kj; ++i)
        if (cfg->job_m[i] > mmax) mmax = cfg->job_m[i];
    if (mmax < 1) mmax = 1;
    int32_t *S = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * z);
    int32_t *Tq = (int32_t *)malloc(sizeof(int32_t) * (size_t)mmax * mmax);
    int32_t *c = (int32_t *)malloc(sizeof(int32_t) * (size_t)mmax);
    int32_t *F0 = (int32_t *)malloc(sizeof(int32_t) * (size_t)mmax);
    uint8_t *y0 = (uint8_t *)malloc((size_t)mmax);
    uint8_t *Y = (uint8_t *)malloc((size_t)mmax * cfg->R);
    int64_t *e = (int64_t *)malloc(sizeof(int64_t) * (size_t)cfg->R);
    uint8_t *inU = (uint8_t *)malloc((size_t)n);
    uint8_t *flip = (uint8_t *)malloc((size_t)n);

    qbo_eta(n, Q, eta);
    qbo_init_x(n, z, cfg->seed, X);
    qbo_field(n, Q, z, X, H);
    qbo_energy(n, z, X, H, E);
    *ebest = INT64_MAX;
    best_update(n, z, X, E, xbest, ebest);
    uint32_t inst = 0;

    if (cfg->init_m > 0 && !cfg->init_jacobi) {
        int m0 = cfg->init_m, L0 = n / m0;
        for (int l = 0; l < L0; ++l) {
            for (int a = 0; a < m0; ++a) S[a] = l * m0 + a;
            for (int p = 0; p < z; ++p) {
                uint8_t *x = X + (int64_t)p * n;
                qbo_extract(n, Q, x, H + (int64_t)p * n, m0, S, Tq, c, F0, y0);
                qbo_anneal(m0, Tq, F0, y0, cfg->nsw_init, cfg->B, cfg->thr_init, cfg->R,
                           cfg->seed, inst + (uint32_t)p, Y, e);
                pick_and_write(m0, S, Y, e, cfg->R, cfg->wb_not_worse, x);
            }
            inst += (uint32_t)z;
            qbo_field(n, Q, z, X, H);
            qbo_energy(n, z, X, H, E);
            best_update(n, z, X, E, xbest, ebest);
        }
    } else if (cfg->init_m > 0) {
        /* the concurrent option: every block of solution p against the
         * state before the pass, job (p, l) numbered p * L0 + l */
        int m0 = cfg->init_m, L0 = n / m0;
        memcpy(X0, X, (size_t)n * z);
        for (int p = 0; p < z; ++p) {
            for (int l = 0; l < L0; ++l) {
                for (int a = 0; a < m0; ++a) S[a] = l * m0 + a;
                qbo_extract(n, Q, X0 + (int64_t)p * n, H + (int64_t)p * n, m0, S, Tq, c, F0, y0);
                qbo_anneal(m0, Tq, F0, y0, cfg->nsw_init, cfg->B, cfg->thr_init, cfg->R, cfg->seed,
                           inst + (uint32_t)(p * L0 + l), Y, e);
                pick_and_write(m0, S, Y, e, cfg->R, cfg->wb_not_worse, X + (int64_t)p * n);
            }
        }
        inst += (uint32_t)(z * L0);
        qbo_field(n, Q, z, X, H);
        qbo_energy(n, z, X, H, E);
        best_update(n, z, X, E, xbest, ebest);
    }

    int t_run = 0, stall = 0;
    for (int t = 0; t < cfg->iters; ++t) {
        const int64_t eprev = *ebest;
        for (int p = 0; p < z; ++p)
            qbo_tabu(n, Q, X + (int64_t)p * n, H + (int64_t)p * n, E + p, cfg->alpha,
                     cfg->tenure, cfg->aspiration, T + (int64_t)p * n, LF + (int64_t)p * n);
        best_update(n, z, X, E, xbest, ebest);

        qbo_keys(n, z, eta, X, T, cfg->W1, cfg->W2, cfg->W3, K);
        if (cfg->random_select) qbo_random_keys(n, z, t, cfg->seed, KR);
        if (learned) {
            qbo_features(n, z, Q, eta, X, H, T, LF, G, cfg->alpha, cfg->scales, F);
            qbo_mlp_scores(n * z, cfg->mlp_W, F, NULL, KL);
        }
        for (int p = 0; p < z; ++p) {
            qbo_order(n, (learned ? KL : cfg->random_select ? KR : K) + (int64_t)p * n, order);
            int off = 0;
            for (int q = 0; q < kj; ++q) {
                int m = cfg->job_m[p * kj + q];
                int32_t *Sq = S + (int64_t)p * n + off;
                memcpy(Sq, order + off, sizeof(int32_t) * (size_t)m);
                qsort(Sq, (size_t)m, sizeof(int32_t), cmp_i32);
                off += m;
            }
        }
        memcpy(X0, X, (size_t)n * z);
        for (int p = 0; p < z && !cfg->no_im; ++p) {
            int off = 0;
            for (int q = 0; q < kj; ++q) {
                int m = cfg->job_m[p * kj + q];
                int32_t *Sq = S + (int64_t)p * n + off;
                qbo_extract(n, Q, X0 + (int64_t)p * n, H + (int64_t)p * n, m, Sq, Tq, c, F0, y0);
                qbo_anneal(m, Tq, F0, y0, cfg->nsw, cfg->B, cfg->thr, cfg->R, cfg->seed,
                           inst + (uint32_t)(p * kj + q), Y, e);
                if (!pick_and_write(m, Sq, Y, e, cfg->R, cfg->wb_not_worse, X + (int64_t)p * n)) {
                    off += m;
                    continue;
                }
                /* last-improvement gain of every variable this job changed */
                int rb = 0;
                for (int r = 1; r < cfg->R; ++r)
                    if (e[r] < e[rb]) rb = r;
                int64_t g = -e[rb];
                if (g > INT32_MAX) g = INT32_MAX;
                if (g < INT32_MIN) g = INT32_MIN;
                for (int a = 0; a < m; ++a)
                    if (Y[(int64_t)rb * m + a] != y0[a]) G[(int64_t)p * n + Sq[a]] = (int32_t)g;
                off += m;
            }
        }
        if (!cfg->no_im) {
            inst += (uint32_t)(z * kj);
            qbo_field(n, Q, z, X, H);
            qbo_energy(n, z, X, H, E);
            best_update(n, z, X, E, xbest, ebest);
        }

        for (int p = 0; p < z; ++p) {
            memset(inU, 0, (size_t)n);
            int tot = 0;
            for (int q = 0; q < kj; ++q) tot += cfg->job_m[p * kj + q];
            if (!cfg->no_im)
                for (int a = 0; a < tot; ++a) inU[S[(int64_t)p * n + a]] = 1;
            if (cfg->random_select)
                qbo_mutate2(n, X + (int64_t)p * n, KR + (int64_t)p * n, K0 + (int64_t)p * n, inU, t, p,
                            cfg->seed, flip);
            else
                qbo_mutate(n, X + (int64_t)p * n, K + (int64_t)p * n, inU, t, p, cfg->seed, flip);
        }
        qbo_field(n, Q, z, X, H);
        qbo_energy(n, z, X, H, E);
        best_update(n, z, X, E, xbest, ebest);
        if (trace_best) trace_best[t] = *ebest;
        t_run = t + 1;
        stall = *ebest < eprev ? 0 : stall + 1;
        if (cfg->patience > 0 && stall >= cfg->patience) break;
    }
    free(eta); free(K0); free(KR); free(T); free(LF); free(G); free(K); free(KL); free(F); free(order); free(X0);
    free(S); free(Tq); free(c); free(F0); free(y0); free(Y); free(e); free(inU); free(flip);
    return t_run;
}

/* ======================================================================== */
/* Learned selector (test infrastructure for the MLP path).
 *
 * Eight per-(solution, variable) features, each an FP32 product of an
 * integer state quantity and a caller-supplied FP32 scale (except Delta, an
 * FP32 quotient), rounded to BF16 with round-to-nearest-even:
 *   0 h_pj sc0   1 Q_jj sc1   2 T_pj sc2   3 age_pj sc3 (age = alpha - LF,
 *   or alpha if never flipped)   4 G_pj sc4 (gain of the last IM job that
 *   changed j)   5 eta_j sc5   6 (z - |2 c_j - z|) sc6   7 (T'_p - T_pj)/T'_p.
 * MLP 8 -> 64 -> 64 -> 1 with ReLU; weights BF16 in the order W1[64][8],
 * b1[64], W2[64][64], b2[64], W3[64], b3 (4801 values); every layer sums in
 * index order in FP32 starting from the bias, hidden activations are rounded
 * to BF16.  Parity status: BF16 rounding pinned against torch's CPU
 * conversion; forward pinned by closed forms and an FP32 reference within
 * rounding; gradients pinned by FP64 central differences. */
uint16_t qbo_bf16_rne(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

float qbo_bf16_to_f32(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

void qbo_features(int n, int z, const int16_t *Q, const int64_t *eta, const uint8_t *X, const int32_t *H,
                  const int32_t *T, const int32_t *LF, const int32_t *G, int alpha, const float *sc, uint16_t *F)
{
    for (int j = 0; j < n; ++j) {
        int32_t cnt = 0;
        for (int p = 0; p < z; ++p) cnt += X[(int64_t)p * n + j];
        int32_t dev = 2 * cnt - z;
        if (dev < 0) dev = -dev;
        for (int p = 0; p < z; ++p) {
            int32_t Tp = 1;
            for (int k = 0; k < n; ++k)
                if (T[(int64_t)p * n + k] > Tp) Tp = T[(int64_t)p * n + k];
            const int64_t at = (int64_t)p * n + j;
            const int32_t age = LF[at] > 0 ? alpha - LF[at] : alpha;
            float f[8];
            f[0] = (float)H[at] * sc[0];
            f[1] = (float)Q[(int64_t)j * n + j] * sc[1];
            f[2] = (float)T[at] * sc[2];
            f[3] = (float)age * sc[3];
            f[4] = (float)G[at] * sc[4];
            f[5] = (float)eta[j] * sc[5];
            f[6] = (float)(z - dev) * sc[6];
            f[7] = (float)(Tp - T[at]) / (float)Tp;
            for (int k = 0; k < 8; ++k) F[at * 8 + k] = qbo_bf16_rne(f[k]);
        }
    }
}

/* offsets of the parameter blocks */
#define QBO_W1 0
#define QBO_B1 512
#define QBO_W2 576
#define QBO_B2 4672
#define QBO_W3 4736
#define QBO_B3 4800
#define QBO_NPARAM 4801

float qbo_mlp_forward(const uint16_t *W, const uint16_t *feat)
{
    float x[8], h1[64], h2[64];
    for (int i = 0; i < 8; ++i) x[i] = qbo_bf16_to_f32(feat[i]);
    for (int k = 0; k < 64; ++k) {
        float acc = qbo_bf16_to_f32(W[QBO_B1 + k]);
        for (int i = 0; i < 8; ++i) acc = acc + qbo_bf16_to_f32(W[QBO_W1 + k * 8 + i]) * x[i];
        h1[k] = qbo_bf16_to_f32(qbo_bf16_rne(acc > 0.0f ? acc : 0.0f));
    }
    for (int k = 0; k < 64; ++k) {
        float acc = qbo_bf16_to_f32(W[QBO_B2 + k]);
        for (int i = 0; i < 64; ++i) acc = acc + qbo_bf16_to_f32(W[QBO_W2 + k * 64 + i]) * h1[i];
        h2[k] = qbo_bf16_to_f32(qbo_bf16_rne(acc > 0.0f ? acc : 0.0f));
    }
    float s = qbo_bf16_to_f32(W[QBO_B3]);
    for (int i = 0; i < 64; ++i) s = s + qbo_bf16_to_f32(W[QBO_W3 + i]) * h2[i];
    return s;
}

/* Order key of a score: larger score -> larger key, -0 and +0 equal. */
int64_t qbo_score_key(float s)
{
    uint32_t u;
    if (s == 0.0f) s = 0.0f;
    memcpy(&u, &s, 4);
    const uint32_t k = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return (int64_t)k - 2147483648LL;
}

void qbo_mlp_scores(int count, const uint16_t *W, const uint16_t *F, float *score, int64_t *K)
{
    for (int e = 0; e < count; ++e) {
        const float s = qbo_mlp_forward(W, F + (int64_t)e * 8);
        if (score) score[e] = s;
        if (K) K[e] = qbo_score_key(s);
    }
}

/* Mean binary cross-entropy of sigmoid(score) against the labels and its
 * gradient with respect to the BF16 parameters.  With round_acts != 0 the
 * forward pass is the FP32 inference pass (BF16 hidden activations) and the
 * backward pass runs in FP64 with the rounding taken as the identity; with
 * round_acts == 0 everything is FP64 (the smooth function the finite
 * differences pin). */
void qbo_mlp_grad(const uint16_t *W, int B, const uint16_t *feat, const uint8_t *label, double *grad,
                  double *loss, int round_acts)
{
    for (int k = 0; k < QBO_NPARAM; ++k) grad[k] = 0.0;
    double L = 0.0;
    for (int b = 0; b < B; ++b) {
        double x[8], z1[64], h1[64], z2[64], h2[64], s;
        for (int i = 0; i < 8; ++i) x[i] = qbo_bf16_to_f32(feat[(int64_t)b * 8 + i]);
        if (round_acts) {
            /* the inference pass itself (FP32, index order, BF16 activations) */
            float xf[8], h1f[64], h2f[64];
            for (int i = 0; i < 8; ++i) xf[i] = (float)x[i];
            for (int k = 0; k < 64; ++k) {
                float acc = qbo_bf16_to_f32(W[QBO_B1 + k]);
                for (int i = 0; i < 8; ++i) acc = acc + qbo_bf16_to_f32(W[QBO_W1 + k * 8 + i]) * xf[i];
                z1[k] = acc;
                h1f[k] = qbo_bf16_to_f32(qbo_bf16_rne(acc > 0.0f ? acc : 0.0f));
                h1[k] = h1f[k];
            }
            for (int k = 0; k < 64; ++k) {
                float acc = qbo_bf16_to_f32(W[QBO_B2 + k]);
                for (int i = 0; i < 64; ++i) acc = acc + qbo_bf16_to_f32(W[QBO_W2 + k * 64 + i]) * h1f[i];
                z2[k] = acc;
                h2f[k] = qbo_bf16_to_f32(qbo_bf16_rne(acc > 0.0f ? acc : 0.0f));
                h2[k] = h2f[k];
            }
            float sf = qbo_bf16_to_f32(W[QBO_B3]);
            for (int i = 0; i < 64; ++i) sf = sf + qbo_bf16_to_f32(W[QBO_W3 + i]) * h2f[i];
            s = sf;
        } else {
            for (int k = 0; k < 64; ++k) {
                double acc = qbo_bf16_to_f32(W[QBO_B1 + k]);
                for (int i = 0; i < 8; ++i) acc += (double)qbo_bf16_to_f32(W[QBO_W1 + k * 8 + i]) * x[i];
                z1[k] = acc;
                h1[k] = acc > 0 ? acc : 0;
            }
            for (int k = 0; k < 64; ++k) {
                double acc = qbo_bf16_to_f32(W[QBO_B2 + k]);
                for (int i = 0; i < 64; ++i) acc += (double)qbo_bf16_to_f32(W[QBO_W2 + k * 64 + i]) * h1[i];
                z2[k] = acc;
                h2[k] = acc > 0 ? acc : 0;
            }
            s = qbo_bf16_to_f32(W[QBO_B3]);
            for (int i = 0; i < 64; ++i) s += (double)qbo_bf16_to_f32(W[QBO_W3 + i]) * h2[i];
        }
        const double y = label[b] ? 1.0 : 0.0;
        /* softplus(s) - y s, computed stably */
        L += (s > 0 ? s + log1p(exp(-s)) : log1p(exp(s))) - y * s;
        const double ds = (1.0 / (1.0 + exp(-s)) - y) / B;
        double dz2[64], dh1[64];
        grad[QBO_B3] += ds;
        for (int i = 0; i < 64; ++i) {
            grad[QBO_W3 + i] += ds * h2[i];
            const double dh2 = ds * qbo_bf16_to_f32(W[QBO_W3 + i]);
            dz2[i] = z2[i] > 0 ? dh2 : 0.0;
        }
        for (int i = 0; i < 64; ++i) dh1[i] = 0.0;
        for (int k = 0; k < 64; ++k) {
            grad[QBO_B2 + k] += dz2[k];
            for (int i = 0; i < 64; ++i) {
                grad[QBO_W2 + k * 64 + i] += dz2[k] * h1[i];
                dh1[i] += dz2[k] * qbo_bf16_to_f32(W[QBO_W2 + k * 64 + i]);
            }
        }
        for (int k = 0; k < 64; ++k) {
            const double dz1 = z1[k] > 0 ? dh1[k] : 0.0;
            grad[QBO_B1 + k] += dz1;
            for (int i = 0; i < 8; ++i) grad[QBO_W1 + k * 8 + i] += dz1 * x[i];
        }
    }
    if (loss) *loss = L / B;
}

/* Initial parameters of the selector MLP (the learned selector is not in the
 * paper; its reading fixes this start).  Weights are uniform on
 * [-a_l, a_l) per layer (a_1 for W1, a_2 for W2, a_3 for W3, passed as FP32
 * constants), biases zero:
 *   u = word (k mod 4) of Philox4x32-10 at counter (k/4, 0, 0, 5<<28), key
 *       the 64-bit seed, for parameter index k;
 *   r = (u >> 8) 2^-24, exactly representable;  w = (2r - 1) a_l, one FP32
 *       rounding;  W = BF16(w), round to nearest even.
 * Pinned in the tests by its range, zero biases, per-layer spread and the
 * uniformity of r. */
void qbo_mlp_init(uint64_t seed, float a1, float a2, float a3, float *master, uint16_t *W)
{
    for (int k = 0; k < QBO_NPARAM; ++k) {
        float a = 0.0f;
        if (k >= QBO_W1 && k < QBO_B1) a = a1;
        else if (k >= QBO_W2 && k < QBO_B2) a = a2;
        else if (k >= QBO_W3 && k < QBO_B3) a = a3;
        float w = 0.0f;
        if (a != 0.0f) {
            const uint32_t u = philox_word((uint32_t)(k >> 2), 0u, 0u, 5u << 28, seed, k & 3);
            const float r = (float)(u >> 8) * (1.0f / 16777216.0f);
            const float c = 2.0f * r - 1.0f;
            w = c * a;
        }
        master[k] = w;
        W[k] = qbo_bf16_rne(w);
    }
}

/* Adam (Kingma & Ba) on FP32 master weights, then the BF16 copy. */
void qbo_adam(int count, float *master, float *m, float *v, const float *grad, int step, float lr,
              float beta1, float beta2, float eps, uint16_t *Wbf)
{
    const float c1 = 1.0f - powf(beta1, (float)step);
    const float c2 = 1.0f - powf(beta2, (float)step);
    for (int k = 0; k < count; ++k) {
        m[k] = beta1 * m[k] + (1.0f - beta1) * grad[k];
        v[k] = beta2 * v[k] + (1.0f - beta2) * grad[k] * grad[k];
        const float mh = m[k] / c1, vh = v[k] / c2;
        master[k] = master[k] - lr * mh / (sqrtf(vh) + eps);
        if (Wbf) Wbf[k] = qbo_bf16_rne(master[k]);
    }
}
