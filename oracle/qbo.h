/*
 * qbo.h -- CPU oracle for the IC-D^2S hot path (TEST INFRASTRUCTURE ONLY).
 *
 * This is a plain, slow, obviously-correct host implementation of every step
 * the GPU library computes.  It is used only by the tests, by the smoke check
 * and by the CPU-baseline leg of the benchmark.  No product code may link,
 * import or call it, and it shares no code (headers, helpers, tables,
 * generators) with the GPU library.
 *
 * Paper: "IC-D^2S: A Hybrid Ising-Classical-Machines Data-Driven QUBO Solver
 * Method" (Abdollahi, Kamal, Pedram, ASP-DAC 2025, arXiv 2502.13947).
 *
 * Conventions (all host memory, row-major):
 *   Q  int16 [n][n], symmetric            eq. 1 objective matrix
 *   X  uint8 [z][n] with values 0/1       the solution set (the paper's S)
 *   H  int32 [z][n]   H[p][i] = sum_j Q[i][j] X[p][j]   (local field)
 *   E  int64 [z]      E[p] = x^T Q x                    (eq. 1)
 *
 * Parity status of each function is stated at its definition in qbo.c.
 */
#ifndef QBO_H
#define QBO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11). */
void qbo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* eq. 1 written out term by term. */
int64_t qbo_energy_def(int n, const int16_t *Q, const uint8_t *x);
/* H = X Q^T (Q symmetric so = X Q). */
void qbo_field(int n, const int16_t *Q, int z, const uint8_t *X, int32_t *H);
/* E[p] = sum_i X[p][i] H[p][i]. */
void qbo_energy(int n, int z, const uint8_t *X, const int32_t *H, int64_t *E);
/* Energy change of flipping variable i of one solution. */
int32_t qbo_flip_delta(int n, const int16_t *Q, const uint8_t *x, const int32_t *h, int i);
/* eta_j = sum_i |Q_ij|  (Weight_Effect_Extraction). */
void qbo_eta(int n, const int16_t *Q, int64_t *eta);

/* sqrt(sum_{i != j} Q_ij^2 / n): the unit of the annealer's temperatures. */
double qbo_sigma(int n, const int16_t *Q);
double qbo_sigma_csr(int n, const int32_t *rowptr, const int32_t *col, const int16_t *val);

/* Initial random solution set (Alg. 2, Generate_Initial_Solution_Set). */
void qbo_init_x(int n, int z, uint64_t seed, uint8_t *X);

/* Tabu search (Alg. 1) on one solution.  x, h updated in place to x_min and
 * its field; *ov in: energy of x, out: OV_min.  T[n] receives flip counts,
 * lastflip[n] the 1-based step of each variable's last flip (0 = never). */
void qbo_tabu(int n, const int16_t *Q, uint8_t *x, int32_t *h, int64_t *ov,
              int alpha, int tenure, int aspiration, int32_t *T, int32_t *lastflip);

/* Control parameters (eta, Delta, gamma) aggregated into exact integer keys
 * K[p][j] = D_p * A[p][j] with D_p > 0 (Alg. 4).  W1..W3 are the weights
 * scaled to integers by a common positive factor. */
void qbo_keys(int n, int z, const int64_t *eta, const uint8_t *X, const int32_t *T,
              int W1, int W2, int W3, int64_t *K);
/* order[r] = index of rank r when sorting by (K desc, index asc). */
void qbo_order(int n, const int64_t *K, int32_t *order);

/* Sub-QUBO of eq. 4 for index set S (m entries, ascending) of one solution.
 * Tq int32 [m][m] (diag 0), c[m] = Q_ii + b_i, F0[m] = local flip basis, y0 = x_S. */
void qbo_extract(int n, const int16_t *Q, const uint8_t *x, const int32_t *h,
                 int m, const int32_t *S, int32_t *Tq, int32_t *c, int32_t *F0, uint8_t *y0);
/* f_S(y) = sum_a c_a y_a + sum_{a != b} T_ab y_a y_b. */
int64_t qbo_sub_energy(int m, const int32_t *Tq, const int32_t *c, const uint8_t *y);

/* Cosine-waveform temperature schedule and its quantised Metropolis threshold
 * table thr[s][b], s < nsw, b < 2^B. */
double qbo_temperature(int s, int nsw, double tmax, double tmin);
void qbo_threshold_table(int nsw, int B, double tmax, double tmin, int32_t *thr);
/* MRAnnealer mutation rate r_t. */
double qbo_mutation_rate(int t);

/* The Ising-machine stage: R replicas of a sequential Metropolis sweep over
 * one sub-QUBO.  Y[R][m] final states, e[R] = f_S(Y_r) - f_S(y0). */
void qbo_anneal(int m, const int32_t *Tq, const int32_t *F0, const uint8_t *y0,
                int nsw, int B, const int32_t *thr, int R, uint64_t seed, uint32_t inst,
                uint8_t *Y, int64_t *e);

void qbo_anneal_count(int m, const int32_t *Tq, const int32_t *F0, const uint8_t *y0,
                      int nsw, int B, const int32_t *thr, int R, uint64_t seed, uint32_t inst,
                      uint8_t *Y, int64_t *e, int32_t *nacc);

/* Ising form (eq. 2, eq. 3) in quarter units: 4 f(x) = E'(2x - 1) + const4
 * with J = -Q off the diagonal (J[n][n], zero diagonal) and h[n]; returns
 * const4.  qbo_ising_energy: E'(s).  qbo_anneal_ising: the spin-form
 * Metropolis sweep (see qbo.c), thr4 in E' units [nsw][2^B]. */
int64_t qbo_ising_from_qubo(int n, const int16_t *Q, int32_t *J, int64_t *h);
int64_t qbo_ising_energy(int n, const int32_t *J, const int64_t *h, const int8_t *s);
void qbo_anneal_ising(int m, const int32_t *J, const int64_t *h, const int8_t *s0, int nsw, int B,
                      const int64_t *thr4, int R, uint64_t seed, uint32_t inst, int8_t *S, int64_t *e);

/* Mutation of one solution p at outer iteration t.  inU[n] marks the
 * variables the IM solved; K the aggregated keys of p.  Flips x in place and
 * writes flip[n] (1 where flipped).  Returns the number of candidates k. */
int qbo_mutate(int n, uint8_t *x, const int64_t *K, const uint8_t *inU, int t, int p,
               uint64_t seed, uint8_t *flip);
/* The same with the candidate order taken from Korder and the flip
 * probabilities from the min-max of Kprob (qbo_mutate uses K for both). */
int qbo_mutate2(int n, uint8_t *x, const int64_t *Korder, const int64_t *Kprob, const uint8_t *inU, int t,
                int p, uint64_t seed, uint8_t *flip);
/* Random keys of the ablation without control parameters (No_SM):
 * K[p][j] = word (j mod 4) of Philox4x32-10 at counter (j/4, t, p, 4<<28). */
void qbo_random_keys(int n, int z, int t, uint64_t seed, int64_t *K);

/* Learned selector (see qbo.c). */
uint16_t qbo_bf16_rne(float f);
float qbo_bf16_to_f32(uint16_t b);
void qbo_features(int n, int z, const int16_t *Q, const int64_t *eta, const uint8_t *X, const int32_t *H,
                  const int32_t *T, const int32_t *LF, const int32_t *G, int alpha, const float *sc, uint16_t *F);
float qbo_mlp_forward(const uint16_t *W, const uint16_t *feat);
int64_t qbo_score_key(float s);
void qbo_mlp_scores(int count, const uint16_t *W, const uint16_t *F, float *score, int64_t *K);
void qbo_mlp_grad(const uint16_t *W, int B, const uint16_t *feat, const uint8_t *label, double *grad,
                  double *loss, int round_acts);
void qbo_mlp_init(uint64_t seed, float a1, float a2, float a3, float *master, uint16_t *W);
void qbo_adam(int count, float *master, float *m, float *v, const float *grad, int step, float lr,
              float beta1, float beta2, float eps, uint16_t *Wbf);

/* Full IC-D^2S run (Alg. 2).  See qbo.c for the exact sequence. */
typedef struct {
    int n, z;
    uint64_t seed;
    int iters;
    int alpha, tenure, aspiration;
    int W1, W2, W3;
    int jobs_per_sol;          /* k */
    const int32_t *job_m;      /* [z][k] sub-QUBO sizes */
    int init_m;                /* initial-pass block size (0 = no initial pass) */
    int nsw_init; const int32_t *thr_init;
    int nsw; int B; const int32_t *thr; int R;
    const uint16_t *mlp_W;     /* NULL: plain selection; else the BF16 MLP picks the IM variables */
    const float *scales;       /* 7 feature scales (learned selection) */
    int random_select;         /* ablation No_SM: random keys instead of the control parameters */
    int no_im;                 /* ablation No_IM: no Ising-machine stage */
    int init_jacobi;           /* initial pass: all blocks against the same state (else one after another) */
    int wb_not_worse;          /* write a sub-solution back only if its energy change is <= 0 */
    int patience;              /* > 0: stop after this many iterations without a better E_best */
} qbo_run_cfg;

/* Outputs: X,H,E final state; xbest[n], *ebest; trace_best[iters] = E_best
 * after each outer iteration run (may be NULL).  Returns the number of outer
 * iterations run, or -1 for an invalid configuration. */
int qbo_run(const int16_t *Q, const qbo_run_cfg *cfg, uint8_t *X, int32_t *H, int64_t *E,
            uint8_t *xbest, int64_t *ebest, int64_t *trace_best);

#ifdef __cplusplus
}
#endif
#endif
