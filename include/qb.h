/*
 * qb.h -- C ABI of the MI355X (gfx950) IC-D^2S hot path.
 *
 * Paper: "IC-D^2S: A Hybrid Ising-Classical-Machines Data-Driven QUBO Solver
 * Method", Abdollahi, Kamal, Pedram (ASP-DAC 2025, arXiv 2502.13947).
 * The method minimises x^T Q x over binary x (eq. 1) by alternating Tabu
 * search (Alg. 1), control-parameter selection (Alg. 4), an Ising-machine
 * stage on extracted sub-QUBOs (eq. 4, Alg. 3) and mutation (Alg. 2).
 *
 * General rules for every call:
 *  - Pointers named *_d are DEVICE pointers owned by the caller; they must
 *    stay valid until the enqueued work completes.  Host pointers are named
 *    *_h.  No call frees or retains caller memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  All
 *    calls only enqueue work on it, except qb_problem_create_dense and
 *    qb_check, which synchronise it.  Results are valid after the stream has
 *    synchronised.
 *  - Every call returns a qb_status; argument errors are detected on the host
 *    before anything is enqueued.  Errors a kernel detects (a value outside a
 *    documented range) are latched in the problem's device status word and
 *    returned by qb_check.  No C++ exception crosses this boundary.
 *  - No call allocates device memory except the handle constructors
 *    qb_problem_create_dense, qb_problem_create_csr, qb_batch_create and
 *    qb_state_create, and the setup-time autotuners qb_autotune_rankk,
 *    qb_autotune_anneal and qb_autotune_anneal_ell.
 *  - Layouts (row-major): Q int16 [n][n] symmetric; X uint8 [z][n] (0/1);
 *    H int32 [z][n] with H[p][i] = sum_j Q[i][j] X[p][j]; E int64 [z].
 *  - Results depend only on inputs, seeds and instance numbers: never on
 *    stream, launch order or occupancy.
 */
#ifndef QB_H
#define QB_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qb_status;
#define QB_OK 0
#define QB_E_ARG (-1)          /* bad pointer, size or flag */
#define QB_E_NOT_SYMMETRIC (-2)/* Q != Q^T (eq. 1 is read as x^T Q x with Q symmetric) */
#define QB_E_RANGE (-3)        /* a value would overflow the int32 field / key packing */
#define QB_E_OVERLAP (-4)      /* jobs of one solution share a variable */
#define QB_E_CAPACITY (-5)     /* size beyond what a kernel supports (see each call) */
#define QB_E_HIP (-6)          /* a HIP runtime call failed; see qb_last_hip_error */
#define QB_E_STATE (-7)        /* a device-side check failed (qb_check) */
#define QB_E_UNSUPPORTED (-8)

typedef struct qb_problem_s *qb_problem;

typedef struct {
    int32_t n;
    int32_t int8_ok;     /* 1 when max |Q_ij| <= 127: an int8 copy of Q is kept */
    int32_t qmax;        /* max |Q_ij| */
    int64_t eta_max;     /* max_j eta_j */
    double sigma;        /* sqrt(sum_{i != j} Q_ij^2 / n): the typical |dE| scale */
    int32_t sparse;      /* 1 for a problem made by qb_problem_create_csr */
    int32_t ell_width;   /* sparse: most off-diagonal entries in one row (>= 1) */
    int32_t tabu_kernel; /* what qb_tabu runs under the problem's Tabu variant: 0 the dense
                            kernel, 1 the sparse lane kernel, 2 the sparse tree kernel
                            (QB_TABU_*), -1 none (n beyond the kernels' capacity) */
} qb_problem_info;

const char *qb_status_str(qb_status s);
/* Last HIP error code seen by this thread (0 if none). */
int32_t qb_last_hip_error(void);
/* Library version string. */
const char *qb_version(void);

/* ---------------------------------------------------------------- problem
 * Eq. 1 input.  Validates symmetry (QB_E_NOT_SYMMETRIC) and the range bound
 * (2n+1) max|Q| < 2^31 that keeps local fields and move values in int32
 * (QB_E_RANGE).  Builds the int8 copy (when |Q| <= 127), eta_j = sum_i |Q_ij|
 * (Weight_Effect_Extraction) and the statistics of qb_problem_info.  The
 * handle BORROWS Q_d (it must outlive the handle) and OWNS its derived
 * buffers.  Synchronises `stream`.  n in [1, 65535]. */
qb_status qb_problem_create_dense(qb_problem *out, int32_t n, const int16_t *Q_d, void *stream);
/* Eq. 1 input in compressed sparse rows (the storage of large sparse
 * instances): rowptr_d int32 [n+1] (rowptr[0] = 0, non-decreasing), col_d
 * int32 [nnz] (strictly ascending within a row, in [0, n)), val_d int16
 * [nnz]; a diagonal entry is optional, a stored zero is allowed.  Checks the
 * structure (QB_E_ARG), symmetry (every (i, j, v) has (j, i, v):
 * QB_E_NOT_SYMMETRIC) and the dense form's range bound (QB_E_RANGE).  The
 * handle COPIES what it needs -- the off-diagonal entries as a row-major
 * ELL of width ell_width (word (v << 16) | j at [i][t]), the diagonal and eta
 * -- so the caller's arrays may be released once the call returns.
 * Synchronises `stream`.  n in [1, 65535]. */
qb_status qb_problem_create_csr(qb_problem *out, int32_t n, const int32_t *rowptr_d, const int32_t *col_d,
                                const int16_t *val_d, void *stream);
void qb_problem_destroy(qb_problem P);
qb_status qb_problem_get_info(qb_problem P, qb_problem_info *info_h);
/* Which kernel qb_tabu runs on a sparse problem (all give the same result):
 * QB_TABU_AUTO the tree kernel where it fits, else the lane kernel;
 * QB_TABU_LANES one 1024-thread workgroup per solution holding the move
 * values in registers, an argmin over all of them per step (n <= 20480);
 * QB_TABU_TREE one wave per solution with the move values in an LDS min-tree
 * of 64-leaf nodes, repairing per step only the nodes the flip touches
 * (n <= 25856 by LDS, ell_width <= 64, 2 dmax < 2^15 - 1 and
 * (2 dmax + 1) 2^ceil(log2 n) < 2^32 with dmax = max|Q_kk| + 2 max eta;
 * qb_tabu returns QB_E_CAPACITY or QB_E_RANGE beyond).  QB_E_ARG for a dense problem or another value. */
#define QB_TABU_AUTO 0
#define QB_TABU_LANES 1
#define QB_TABU_TREE 2
qb_status qb_problem_set_tabu_variant(qb_problem P, int32_t variant);
/* Copies eta (int64 [n]) into eta_d. */
qb_status qb_problem_eta(qb_problem P, int64_t *eta_d, void *stream);
/* Synchronises `stream` and returns QB_E_STATE if any kernel latched an error
 * since the last qb_check (the latch is then cleared), else QB_OK. */
qb_status qb_check(qb_problem P, void *stream);

/* ---------------------------------------------------------------- a1
 * Generate_Initial_Solution_Set (Alg. 2): X[p][j] = top bit of Philox4x32-10
 * word (j mod 4) at counter (j/4, p, 0, 3<<28), key (seed lo, seed hi). */
qb_status qb_init_solutions(int32_t n, int32_t z, uint64_t seed, uint8_t *X_d, void *stream);

/* ---------------------------------------------------------------- a0/a8
 * Local field H = X Q (all z solutions, from scratch). */
qb_status qb_field(qb_problem P, int32_t z, const uint8_t *X_d, int32_t *H_d, void *stream);
/* Exact energy E[p] = sum_i X[p][i] H[p][i] = x^T Q x (eq. 1), int64. */
qb_status qb_energy(int32_t n, int32_t z, const uint8_t *X_d, const int32_t *H_d, int64_t *E_d,
                    void *stream);
/* Best tracking (Alg. 1/2 x_min, OV_min): for p = 0..z-1 in order, if
 * E[p] < *ebest_d then *ebest_d = E[p] and xbest_d = X[p].  Initialise
 * *ebest_d to INT64_MAX before the first call. */
qb_status qb_best(int32_t n, int32_t z, const uint8_t *X_d, const int64_t *E_d, int64_t *ebest_d,
                  uint8_t *xbest_d, void *stream);

/* ---------------------------------------------------------------- a2
 * Tabu search (Alg. 1) on every solution, in place.  Move value of k is the
 * exact energy change Q_kk + 2(1-2x_k)h_k; each of `alpha` steps flips the
 * lowest-index argmin among variables whose tenure counter is <= 0 or, when
 * `aspiration` != 0, whose move reaches OV + move < OV_min (if none is
 * allowed, the argmin over all); then C_i += tenure and every positive C is
 * decremented.  On return X[p] = x_min, H[p] = Q x_min, E[p] = OV_min
 * (E[p] must hold x^T Q x on entry), T[p][j] = flips of j, LF[p][j] = the
 * 1-based step of j's last flip (0 if none).  A tenure beyond alpha + 1
 * is taken as alpha + 1 (the same search).  Capacity: n <= 16384 (dense
 * problems; one workgroup of 512 or 1024 threads per solution, fixed when
 * the problem is created from n and the range of the move values, every
 * step reads one row of Q) or, for sparse problems (every step reads the
 * flipped variable's off-diagonal entries only), n <= 25856 on the tree
 * kernel and n <= 20480 on the lane kernel (qb_problem_set_tabu_variant);
 * QB_E_CAPACITY beyond.  QB_E_RANGE when |Q_kk| + 2 max_k eta_k
 * leaves too few bits for the kernel's 32-bit (move, element) keys.  T_d
 * and LF_d may not be NULL. */
qb_status qb_tabu(qb_problem P, int32_t z, uint8_t *X_d, int32_t *H_d, int64_t *E_d,
                  int32_t alpha, int32_t tenure, int32_t aspiration, int32_t *T_d, int32_t *LF_d,
                  void *stream);

/* ---------------------------------------------------------------- a3
 * Control parameters (eta, Delta, gamma) aggregated per Alg. 4 as exact
 * integer keys with the same order as A within each solution:
 *   K[p][j] = W1 eta_j z T'_p + W2 (z - |2 c_j - z|) eta_max T'_p
 *             - W3 (T'_p - T[p][j]) eta_max z,
 * c_j = sum_p X[p][j], T'_p = max(max_j T[p][j], 1), i.e. A scaled by
 * eta_max z T'_p with weights (W1, W2, W3) / common denominator (Table 1's
 * (1, 1, 0.5) is (2, 2, 1)).  T entries must be in [0, t_bound]; QB_E_RANGE
 * if (W1+W2+W3) eta_max z max(t_bound,1) >= 2^47 (the rank packing). */
qb_status qb_keys(qb_problem P, int32_t z, const uint8_t *X_d, const int32_t *T_d, int32_t W1,
                  int32_t W2, int32_t W3, int32_t t_bound, int64_t *K_d, void *stream);
/* Random keys for the ablation that omits the control parameters (No_SM of
 * the Discussion section): K[p][j] = word (j mod 4) of Philox4x32-10 at
 * counter (j/4, t, p, 4<<28), key (seed lo, seed hi), as int64 in [0, 2^32).
 * Ranked by qb_rank like the plain keys, they pick the sub-QUBO variables
 * and order the mutation candidates at random. */
qb_status qb_random_keys(int32_t n, int32_t z, int32_t t, uint64_t seed, int64_t *K_d, void *stream);
/* order[p][r] = variable of rank r when sorting solution p by (K desc, index
 * asc) (Alg. 3 "highest values in A"; ties to the lower index).  Keys must
 * satisfy |K| < 2^47 (guaranteed by qb_keys).  n <= 16384 sorts in LDS;
 * larger n (up to 65535) sorts indices in place in order_d with only the
 * short strides in LDS. */
qb_status qb_rank(int32_t n, int32_t z, const int64_t *K_d, int32_t *order_d, void *stream);

/* ---------------------------------------------------------------- jobs
 * A batch of J sub-QUBO jobs (the multi-IM fabric of Alg. 3: several
 * sub-QUBOs per solution solved at once).  Job q belongs to solution sol[q]
 * (sol non-decreasing: the jobs of one solution are consecutive) and has
 * m_q = size[q] variables; its index set idx[off[q] .. off[q+1]) is stored
 * ascending, off being the prefix sum of the sizes.  rank0[q] is the first
 * rank of qb_rank's order the job takes (NULL = consecutive chunks from rank
 * 0 per solution, in job order).  The handle OWNS its device metadata (sol,
 * off, rank0, idx, tile offsets, dispatch order) and the side streams used to
 * run the annealer's size classes concurrently; create/destroy are not hot
 * calls.  Capacity: 1 <= m_q <= 1024, sum of a solution's sizes <= n.
 * J = 0 makes an empty batch (sol_h and size_h may be NULL): every per-job
 * call returns at once, and qb_mutate sees no IM variables (U_p empty). */
typedef struct qb_batch_s *qb_batch;
typedef struct {
    int32_t J;
    int32_t total;            /* off[J] */
    int32_t m_max;
    int64_t tile_elems;       /* elements a tile buffer for qb_extract needs */
    const int32_t *sol_d;     /* [J] */
    const int32_t *off_d;     /* [J+1] */
    int32_t *idx_d;           /* [total] */
    int64_t dblk_words;       /* words after the ELL rows in a qb_extract_ell tile buffer */
} qb_batch_info;

/* Result-invariant schedule of qb_anneal on a batch (qb_autotune_anneal
 * picks one; every plan gives the same Y and e):
 *   sleep_after: polls of a list word not yet written before a waiting wave
 *     sleeps between polls (0: at once);
 *   depth: list words a wave that reads rows from global memory keeps in
 *     flight (8, 16 or 32);
 *   kernel[c]: the kernel of size class c (c = 0..4 for padded widths
 *     mp = 1024, 512, 256, 128, 64): QB_ANNEAL_AUTO (a replica spread over
 *     up to four waves where its replicas fit one workgroup, else one wave
 *     per replica), QB_ANNEAL_MULTI_WAVE, QB_ANNEAL_ONE_WAVE, or
 *     QB_ANNEAL_ONE_WAVE_REG (one wave per replica holding the current
 *     diagonal block's couplings in registers; tiles in LDS only: int8
 *     mp <= 512, int16 mp <= 128), or QB_ANNEAL_MULTI_WAVE_GLOBAL (a
 *     replica over up to four waves reading the tile rows from global memory,
 *     a few KB of LDS, so that several jobs share a compute unit; R = 1); a
 *     kernel that cannot run the class falls back to the automatic choice;
 *   persistent: 1 = each class runs as a persistent grid of
 *     wgs_per_cu workgroups per compute unit (at most one per job) that pull
 *     the class's jobs from an atomic queue; 0 = one workgroup per job;
 *   lpt: the queue (and dispatch) order within a class: 1 = largest job
 *     first (longest processing time), 0 = job index order.
 * Size classes run concurrently (their own streams, joined back into the
 * caller's). */
#define QB_ANNEAL_AUTO 0
#define QB_ANNEAL_MULTI_WAVE 1
#define QB_ANNEAL_ONE_WAVE 2
#define QB_ANNEAL_ONE_WAVE_REG 3
#define QB_ANNEAL_MULTI_WAVE_GLOBAL 4
typedef struct {
    int32_t sleep_after;
    int32_t depth;
    int32_t kernel[5];
    int32_t persistent;
    int32_t wgs_per_cu;
    int32_t lpt;
} qb_anneal_plan;
qb_status qb_batch_set_anneal_plan(qb_batch b, const qb_anneal_plan *plan_h);
qb_status qb_batch_get_anneal_plan(qb_batch b, qb_anneal_plan *plan_h);
qb_status qb_batch_create(qb_batch *out, int32_t n, int32_t z, int32_t J, const int32_t *sol_h,
                          const int32_t *size_h, const int32_t *rank0_h);
void qb_batch_destroy(qb_batch b);
qb_status qb_batch_get_info(qb_batch b, qb_batch_info *info_h);
/* Host-provided index sets (e.g. the contiguous blocks of the initial pass):
 * validated on the host (ascending within a job, in [0,n), disjoint within a
 * solution: QB_E_ARG / QB_E_OVERLAP), then copied to the handle's idx. */
qb_status qb_batch_set_idx(qb_batch b, const int32_t *idx_h, void *stream);
/* Synchronises `stream` and returns QB_E_STATE if, since the last
 * qb_batch_check, qb_writeback met a job with a replica that did not finish
 * (e = INT64_MIN, see qb_set_anneal_wait_limit); the latch is then cleared.
 * Such replicas are never chosen: a job none of whose replicas finished is
 * not written back (qb_writeback), gives no gain (qb_gain_update) and no
 * positive label (qb_trace). */
qb_status qb_batch_check(qb_batch b, void *stream);
/* Measurement hook: with acnt_d (device int32 [J * R], caller-owned) set,
 * every later qb_anneal / qb_anneal_ell on the batch also writes the number
 * of accepted moves of replica r of job q to acnt_d[q * R + r] (the count
 * that sets the annealer's row traffic); NULL turns it off.  Results are
 * unchanged. */
qb_status qb_batch_count_accepts(qb_batch b, int32_t *acnt_d);
/* Copies the handle's index sets (int32 [total]) into idx_d. */
qb_status qb_batch_copy_idx(qb_batch b, int32_t *idx_d, void *stream);

/* Plain selection (the selection step of Alg. 3): job q takes the ranks [rank0[q],
 * rank0[q] + m_q) of its solution in order_d and stores their indices
 * ascending in the handle's idx. */
qb_status qb_select(qb_batch b, const int32_t *order_d, void *stream);

/* ---------------------------------------------------------------- a4
 * Sub-QUBO extraction, eq. 4 / the sub-QUBO construction of Alg. 3, against the state (X, H).
 * For job q with S = idx of q, m = m_q, MS = the power of two >= ceil(m/64)
 * (1, 2, 4, 8 or 16) and mp = 64 MS:
 *   tile  (int8 if the problem is int8_ok, else int16), element
 *         [tile_off[q] + a*mp + L*MS + s] = T[a][64 s + L] with
 *         T[a][b] = Q[S_a][S_b] for a != b, 0 on the diagonal and padding;
 *         tile_off is the prefix sum of mp^2 over the jobs (the buffer holds
 *         qb_batch_info.tile_elems elements, 16-byte aligned);
 *   c[off[q]+a]  = Q_aa + b_a,  b_a = 2 sum_{j not in S} Q[S_a][j] x_j;
 *   F0[off[q]+a] = c_a + 2 sum_{b != a} T[a][b] y0_b (flip basis);
 *   y0[off[q]+a] = X[p][S_a].
 * c_d may be NULL.  Dense problems only (QB_E_UNSUPPORTED for a sparse one:
 * use qb_extract_ell). */
qb_status qb_extract(qb_problem P, qb_batch b, const uint8_t *X_d, const int32_t *H_d,
                     void *tile_d, int32_t *c_d, int32_t *F0_d, uint8_t *y0_d, void *stream);

/* ---------------------------------------------------------------- a5
 * The Ising-machine stage on every job at once: R replicas of a sequential
 * Metropolis sweep (positions 0..m-1 in order, nsw sweeps), warm-started at
 * y0 with flip basis F0.  The uniform of (replica r, sweep s, position k) is
 * word ((k>>6)&3) of Philox4x32-10 at counter (((k>>8)<<6)|(k&63), s, r,
 * (1<<28)|(inst_base+q)), key (seed lo, seed hi); the move (1-2y_k) F_k is
 * accepted iff it is <= thr[s][u >> (32-B)].  Outputs, per job q, replica r:
 *   Y[off[q]*R + r*m_q + k] final state, e[q*R + r] = f_S(Y_r) - f_S(y0).
 * thr_d: int32 [nsw][2^B] (see qb_threshold_table).  tile as qb_extract;
 * int8_tile selects its element type.  Jobs are grouped by padded size and
 * the groups run concurrently (side streams joined back into `stream`),
 * largest first.  The tile must be symmetric (as qb_extract writes it).
 * Capacity: 1 <= R <= 16, 1 <= B <= 16, nsw >= 1, inst_base + J <= 2^28.
 * Where a replica's sweep is spread over several waves of a workgroup, the
 * waves wait on each other with bounded waits (qb_set_anneal_wait_limit); a
 * replica whose wait runs out (never seen at the default limit) reports
 * e = INT64_MIN, so every launch completes. */
qb_status qb_anneal(qb_batch b, const void *tile_d, int32_t int8_tile, const int32_t *F0_d,
                    const uint8_t *y0_d, int32_t nsw, int32_t B, const int32_t *thr_d, int32_t R,
                    uint64_t seed, uint32_t inst_base, uint8_t *Y_d, int64_t *e_d, void *stream);
/* Bounds the waits between the waves of one replica in the multi-wave
 * annealers (qb_anneal): a wave that reads a list word `polls` times without
 * finding it written gives up, and its replica reports e = INT64_MIN (Y then
 * holds an unfinished state).  Default 2^24 polls (about a second); 0 makes
 * every wait that does not succeed at once give up.  Process-wide, takes
 * effect at the next launch; for tests of that path.  QB_E_ARG if polls < 0. */
qb_status qb_set_anneal_wait_limit(int32_t polls);

/* Sparse sub-QUBOs (eq. 4 on a problem made by qb_problem_create_csr).  Same
 * c, F0 and y0 as qb_extract; the tile is an ELL of width W = ell_width:
 * uint32 word [off[q]*W + a*W + t] = (T[a][b] << 16) | b for the t-th
 * non-zero T[a][b] (b != a, ascending b) of row a, zero words after the last
 * one.  For a problem with |Q| <= 127 the jobs' diagonal 64 x 64 blocks
 * follow the rows as int8 (dblk_words = 1024 words per block, qb_tile_ms(m)
 * blocks per job in job order; byte [block][L][k] = T[64 b + k][64 b + L],
 * zero outside the job), which qb_anneal_ell keeps in registers.  The
 * buffer holds off[J]*W + dblk_words words, 16-byte aligned. */
qb_status qb_extract_ell(qb_problem P, qb_batch b, const uint8_t *X_d, const int32_t *H_d, uint32_t *tile_d,
                         int32_t *c_d, int32_t *F0_d, uint8_t *y0_d, void *stream);
/* qb_anneal on ELL tiles (qb_extract_ell, width W): the same sweep, the same
 * random numbers and thresholds, bit-identical results (Y, e).  rw replicas
 * share a workgroup and its tile copy (1 <= rw <= 16; 0 = automatic); rw only
 * changes the schedule, never the result.  Capacity as qb_anneal, and
 * m_q * W + rw * 64 * ceil(m_q/64) words must fit the 160 KiB of LDS of one
 * workgroup (QB_E_CAPACITY). */
qb_status qb_anneal_ell(qb_batch b, int32_t W, const uint32_t *tile_d, const int32_t *F0_d, const uint8_t *y0_d,
                        int32_t nsw, int32_t B, const int32_t *thr_d, int32_t R, int32_t rw, uint64_t seed,
                        uint32_t inst_base, uint8_t *Y_d, int64_t *e_d, void *stream);

/* The IM stage in Ising form (eq. 2, eq. 3), the native input of hardware
 * Ising machines.  Job q is given as couplings J_q in the tile layout of
 * qb_extract (element [tile_off[q] + a*mp + L*MS + s] = J[a][64s+L], J
 * symmetric; diagonal and padding ignored; int8 or int16 as int8_tile
 * says), fields h_d (int32 [total]) and start spins s0_d (int8 [total], -1
 * or +1), and annealed on E'(s) = -sum_{a != b} J_ab s_a s_b - sum_a h_a s_a
 * with the sweep, uniforms and replica layout of qb_anneal: the move of
 * spin k is E'(s with s_k flipped) - E'(s), accepted iff <= thr[s][u >>
 * (32-B)] (thr_d in E' units).  Outputs S_d (int8 [total*R], spins, layout
 * of Y) and e_d (int64 [J*R]) = E'(S_r) - E'(s0).  For the Ising form of a
 * QUBO (J = -Q off the diagonal, h_i = -2 (Q_ii + sum_{j != i} Q_ij): then
 * 4 f(x) = E'(2x - 1) + const) and thresholds 4 thr, the result is
 * qb_anneal's (S = 2Y - 1, e' = 4e).  A job with an asymmetric J, |J| >
 * 8191, a spin not in {-1, +1} or a start field |2 sum_b J_ab s0_b + h_a| >=
 * 2^30 is not
 * annealed: its spins stay s0 and every e of it is INT64_MIN.  work_d:
 * qb_anneal_ising_workspace(b, R) bytes, 256-byte aligned, owned by the
 * caller.  Capacity as qb_anneal. */
size_t qb_anneal_ising_workspace(qb_batch b, int32_t R);
qb_status qb_anneal_ising(qb_batch b, const void *J_tile_d, int32_t int8_tile, const int32_t *h_d,
                          const int8_t *s0_d, int32_t nsw, int32_t B, const int32_t *thr_d, int32_t R,
                          uint64_t seed, uint32_t inst_base, void *work_d, int8_t *S_d, int64_t *e_d,
                          void *stream);

/* Host builder of the acceptance table (cosine-waveform temperature, the
 * MRAnnealer's waveform used as the IM temperature schedule):
 *   T_s = tmin + 0.5 (tmax - tmin)(1 + cos(pi s / (nsw - 1)))   (T_0 = tmax
 *   when nsw == 1), thr[s][b] = floor(T_s (-ln((b + 1/2) / 2^B))) capped at
 *   2^31 - 1.  thr_h: host int32 [nsw][2^B]. */
qb_status qb_threshold_table(int32_t nsw, int32_t B, double tmax, double tmin, int32_t *thr_h);

/* ---------------------------------------------------------------- a6/a7/a8
 * Write-back (the last step of Alg. 3): per job the replica with the lowest e (lowest
 * r on ties; replicas reporting e = INT64_MIN did not finish and are skipped,
 * a job with none left is not written back and its ebest_job is INT64_MIN,
 * and the batch latches QB_E_STATE for qb_batch_check) is written into
 * X[sol][S] unconditionally, and dX[sol][S] = Y - y0 (int8 in {-1,0,1}).  flags bit 0 (QB_WB_NOT_WORSE): write a job
 * back only if that e <= 0 (the "only if not worse" variant; otherwise X
 * and dX of the job are left untouched).  dX_d (int8 [z][n]) must be all
 * zero on entry outside the jobs' variables.  ebest_job_d (optional, int64
 * [J]) receives the chosen e.  Jobs of one solution are disjoint (qb_select
 * builds them so; qb_batch_set_idx checks it). */
#define QB_WB_NOT_WORSE 1
qb_status qb_writeback(qb_batch b, int32_t R, const uint8_t *Y_d, const int64_t *e_d,
                       const uint8_t *y0_d, uint8_t *X_d, int8_t *dX_d, int64_t *ebest_job_d,
                       int32_t flags, void *stream);
/* Rank-k local-field update H[p] += Q dX[p] for all p (the O(n) move-value
 * update of the Tabu section generalised to many flipped variables).
 * variant: 0 = automatic, 1 = VALU gather over the changed columns,
 * 2 = int8 MFMA dense contraction (int8_ok problems only), 3 = ELL sparse
 * product (the only variant of a sparse problem).  Exact (int32). */
qb_status qb_rankk(qb_problem P, int32_t z, const int8_t *dX_d, int32_t *H_d, int32_t variant,
                   void *stream);
/* Fill an int8 buffer with zeros (a kernel, safe under graph capture). */
qb_status qb_zero(void *buf_d, size_t bytes, void *stream);

/* ---------------------------------------------------------------- a9
 * Mutation (end of the heuristic section).  For every solution p the
 * candidates are the variables not solved by the IM (not in any job of p);
 * the first k_p = floor((n - |U_p|) * rate) of them in qb_rank order are
 * flipped with probability P_j = min(floor(2^32 (K_j - K_lo)/(K_hi - K_lo)),
 * 2^32-1) (2^31 when K_hi == K_lo; K_lo/K_hi the min/max of K[p]); the flip
 * happens iff word (j mod 4) of Philox4x32-10 at counter (j/4, t, p, 2<<28)
 * is < P_j.  rate is r_t of the MRAnnealer (qb_mutation_rate).  X updated in
 * place; dX (all zero on entry) receives the +-1 changes; kcount_d
 * (optional, int32 [z]) receives k_p.  Solutions without jobs in the batch
 * have U_p empty.  Capacity: n <= 65535. */
qb_status qb_mutate(qb_batch b, const int64_t *K_d, const int32_t *order_d, double rate,
                    int32_t t, uint64_t seed, uint8_t *X_d, int8_t *dX_d, int32_t *kcount_d,
                    void *stream);
/* r_t = 0.3 (1 + cos(pi t / 15)) 0.99^t. */
double qb_mutation_rate(int32_t t);

/* ---------------------------------------------------------------- a3' / a10
 * Learned selection.  An MLP scores every (solution, variable) and the top
 * scores go to the annealer instead of the top control-parameter values;
 * the plain keys still drive the mutation, and the exact integer energy still
 * decides every result, so the network only changes which variables are
 * chosen, never the arithmetic.
 *
 * qb_features: eight features per (p, j), each an FP32 product of an integer
 * state quantity and a caller-supplied FP32 scale, rounded to BF16 (round to
 * nearest even), stored F[p][j][0..7] (uint16 BF16 bits, 16-byte aligned):
 *   0 H[p][j] sc0    1 Q_jj sc1    2 T[p][j] sc2 (Tabu flips)
 *   3 age sc3, age = alpha - LF[p][j] if LF > 0 else alpha (Tabu steps since
 *     the last flip)   4 G[p][j] sc4 (gain of the last IM job that changed j,
 *     see qb_gain_update)   5 eta_j sc5   6 (z - |2 c_j - z|) sc6 (gamma z)
 *   7 (T'_p - T[p][j]) / T'_p, T'_p = max(max_j T[p][j], 1) (Delta).
 * scales_h: host float[7] (sc0..sc6). */
qb_status qb_features(qb_problem P, int32_t z, const uint8_t *X_d, const int32_t *H_d, const int32_t *T_d,
                      const int32_t *LF_d, const int32_t *G_d, int32_t alpha, const float *scales_h,
                      uint16_t *F_d, void *stream);
/* MLP 8 -> 64 -> 64 -> 1 with ReLU; W_d holds 4801 BF16 parameters in the
 * order W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3.  Each layer sums in
 * index order in FP32 from its bias; hidden activations are rounded to BF16.
 * For each of `count` feature rows: score_d (optional, float) and the order
 * key K_d (int64, larger score -> larger key, -0 == +0), which qb_rank and
 * qb_select consume like the plain keys. */
qb_status qb_mlp_score(int64_t count, const uint16_t *F_d, const uint16_t *W_d, float *score_d, int64_t *K_d,
                       void *stream);
/* Improvement traces: for every job variable a, outF[off[q]+a] = F[sol][S_a]
 * and outL[off[q]+a] = 1 iff the chosen replica changed it and lowered the
 * sub-QUBO energy (e < 0). */
qb_status qb_trace(qb_batch b, int32_t R, const uint16_t *F_d, const uint8_t *Y_d, const int64_t *e_d,
                   const uint8_t *y0_d, uint16_t *outF_d, uint8_t *outL_d, void *stream);
/* G[sol][S_a] = -e (saturated to int32) of the chosen replica for every
 * variable the job changed. */
qb_status qb_gain_update(qb_batch b, int32_t R, const uint8_t *Y_d, const int64_t *e_d, const uint8_t *y0_d,
                         int32_t *G_d, void *stream);
/* Mean binary cross-entropy of sigmoid(score) against the labels over B
 * samples and its gradient (float [4801]) with respect to the parameters.
 * The forward pass rounds as the inference pass does (BF16 activations,
 * FP32 sums); the three 64 x 64 products of the second layer (forward, the
 * backward into the first layer, and the W2 gradient) run on the matrix
 * cores with BF16 operands and FP32 accumulation, the output gradient dZ2
 * entering them as a BF16 pair hi + lo.  So the loss and the activations
 * agree with qb_mlp_score up to the summation order of the second layer (an
 * activation can round to the neighbouring BF16 value).  The BF16 rounding
 * is taken as the identity backward; per-64-sample partial sums are added in
 * a fixed order (deterministic: the same inputs give the same bits).
 * work_d: qb_mlp_train_workspace(B) bytes. */
size_t qb_mlp_train_workspace(int32_t B);
qb_status qb_mlp_grad(int32_t B, const uint16_t *feat_d, const uint8_t *label_d, const uint16_t *W_d,
                      float *grad_d, float *loss_d, void *work_d, void *stream);
/* qb_mlp_grad for callers that cannot allocate (code under HIP graph
 * capture, tight training loops, harnesses that forbid allocation): the
 * same kernels and the same result, bit for bit, with the per-workgroup
 * partial sums in a static device array of the library (one per GPU, about
 * 2.4 MB, held until the process ends) instead of a workspace.  B up to
 * QB_MLP_GRAD_NOALLOC_MAX_B (QB_E_CAPACITY beyond).  Calls that overlap on
 * one GPU share that array and race; calls on one stream do not.  Allocates
 * nothing (the array's device address is looked up on the first call on
 * each device). */
#define QB_MLP_GRAD_NOALLOC_MAX_B 8192
qb_status qb_mlp_grad_noalloc(int32_t B, const uint16_t *feat_d, const uint8_t *label_d, const uint16_t *W_d,
                              float *grad_d, float *loss_d, void *stream);
/* Initial parameters of the MLP (the learned selector is this library's
 * addition to the method, so its start is this library's choice): weights
 * uniform on [-a_l, a_l) for W1, W2, W3 (a1, a2, a3), biases zero.
 * Parameter k draws word (k mod 4) of Philox4x32-10 at counter
 * (k/4, 0, 0, 5<<28), key (seed lo, seed hi); r = (u >> 8) 2^-24 and
 * master[k] = (2r - 1) a_l in FP32 (one rounding), W_d[k] = BF16(master[k])
 * (round to nearest even).  master_d float [4801], W_d uint16 [4801]. */
qb_status qb_mlp_init(uint64_t seed, float a1, float a2, float a3, float *master_d, uint16_t *W_d, void *stream);
/* Adam on FP32 master weights (count 4801), then W_d = BF16(master). */
qb_status qb_mlp_adam(const float *grad_d, float *master_d, float *m_d, float *v_d, int32_t step, float lr,
                      float beta1, float beta2, float eps, uint16_t *W_d, void *stream);

/* ---------------------------------------------------------------- a11
 * Outer-loop orchestration (Alg. 2).  Work the caller enqueues on `stream`
 * (a non-default stream) between qb_graph_begin and qb_graph_end -- e.g. a
 * fixed number of outer iterations, with every per-iteration scalar (t, r_t,
 * instance numbers) baked into the launches -- becomes one executable HIP
 * graph; qb_graph_launch replays it.  Capture uses relaxed mode and follows
 * the annealer's side streams.  The handle is owned by the caller
 * (qb_graph_destroy). */
qb_status qb_graph_begin(void *stream);
qb_status qb_graph_end(void *stream, void **graph_exec_out);
qb_status qb_graph_launch(void *graph_exec, void *stream);
void qb_graph_destroy(void *graph_exec);
/* Autotuner for the result-invariant rank-k variants: times each applicable
 * variant `reps` times on (dX, H) (H unchanged on return), checks that all of
 * them produce the same field (else QB_E_STATE), and returns the fastest in
 * *variant_out (its mean time in *ms_out if not NULL).  Not a hot call: it
 * allocates scratch and synchronises `stream`. */
qb_status qb_autotune_rankk(qb_problem P, int32_t z, const int8_t *dX_d, const int32_t *H_d, int32_t reps,
                            int32_t *variant_out, float *ms_out, void *stream);
/* Plan autotuner of qb_anneal (the batching schedule): coordinate descent
 * over qb_anneal_plan on the given jobs -- the kernel of each size class
 * present (largest first), the persistent job queue with its grid
 * (workgroups per compute unit) and its order (longest job first or job
 * order), and the consumers' loads in flight -- timing `reps` launches of
 * each candidate after a warm-up launch.  Every candidate must give the same
 * Y and e as the batch's plan on entry (else QB_E_STATE).  The fastest plan
 * is left set on the batch and returned in *plan_out (its mean time in
 * *ms_out; both optional).  Not a hot call: it allocates scratch and
 * synchronises `stream`. */
qb_status qb_autotune_anneal(qb_batch b, const void *tile_d, int32_t int8_tile, const int32_t *F0_d,
                             const uint8_t *y0_d, int32_t nsw, int32_t B, const int32_t *thr_d, int32_t R,
                             uint64_t seed, uint32_t inst_base, int32_t reps, qb_anneal_plan *plan_out, float *ms_out,
                             void *stream);
/* Autotuner for qb_anneal_ell's replicas per workgroup: times rw in
 * {1, 2, 4, 8, 16} (those <= R that fit LDS) `reps` times each on the given
 * jobs, checks that every rw gives the same Y and e (else QB_E_STATE), and
 * returns the fastest in *rw_out (its mean time in *ms_out if not NULL).  Not
 * a hot call: it allocates scratch and synchronises `stream`. */
qb_status qb_autotune_anneal_ell(qb_batch b, int32_t W, const uint32_t *tile_d, const int32_t *F0_d,
                                 const uint8_t *y0_d, int32_t nsw, int32_t B, const int32_t *thr_d, int32_t R,
                                 uint64_t seed, uint32_t inst_base, int32_t reps, int32_t *rw_out, float *ms_out,
                                 void *stream);

/* ---------------------------------------------------------------- a11 / b: state
 * The main loop of Alg. 2 inside the library.  A qb_state holds one run of
 * the method on a problem: the solution set and its fields, energies and
 * Tabu statistics, the keys and orders of the selection, the sub-QUBO
 * batch with its tiles and annealer outputs, the best solution, the
 * per-iteration E_best trace and a device record of the iteration number
 * and annealer instance, so that one captured outer iteration replays
 * every later one.  Each buffer of qb_state_buffers given non-NULL at
 * creation is BORROWED (caller-owned device memory of the stated size,
 * which must outlive the state); the others are allocated and OWNED by the
 * state.  Creation and destruction are not hot calls; qb_state_init,
 * qb_iterate and qb_apply allocate nothing.
 *
 * One outer iteration (Alg. 2, in this order on `stream`):
 *   Tabu (Alg. 1) on every solution, best;
 *   keys (Alg. 4), rank; selection: the top control-parameter values
 *     (plain), the top MLP scores of the features (QB_RUN_LEARNED) or random
 *     keys (QB_RUN_RANDOM_SELECT, the No_SM ablation);
 *   unless QB_RUN_NO_IM: extraction (eq. 4), the annealer (instance numbers
 *     continuing from the previous iteration), gains and traces when kept,
 *     write-back (Alg. 3), rank-k field update, energy, best;
 *   mutation with r_t of the MRAnnealer, field update, energy, best;
 *   E_best recorded for the iteration; iteration number advanced. */
typedef struct qb_state_s *qb_state;
#define QB_RUN_RANDOM_SELECT 1   /* No_SM ablation: random keys rank the IM variables and mutation candidates */
#define QB_RUN_NO_IM 2           /* No_IM ablation: no Ising-machine stage */
#define QB_RUN_INIT_JACOBI 4     /* initial pass: all blocks against one state (else block after block) */
#define QB_RUN_WB_NOT_WORSE 8    /* write a sub-solution back only if its e <= 0 */
#define QB_RUN_LEARNED 16        /* the MLP (mlp_W_d) picks the IM variables */
typedef struct {
    int32_t z;                  /* solutions, >= 1 */
    int32_t k;                  /* sub-QUBO jobs per solution, >= 1 */
    const int32_t *job_m_h;     /* host int32 [z][k] job sizes (1..1024, sum per solution <= n) */
    uint64_t seed;              /* key of every Philox stream of the run */
    int32_t init_m;             /* block size of the initial pass (Call_IM_Solution_Set); 0 = none */
    int32_t nsw_init;           /* sweeps of the initial pass (>= 1 when init_m > 0) */
    const int32_t *thr_init_h;  /* host int32 [nsw_init][2^B] acceptance table of the initial pass */
    int32_t nsw;                /* sweeps of the IM stage */
    const int32_t *thr_h;       /* host int32 [nsw][2^B] acceptance table of the IM stage */
    int32_t B;                  /* table index bits (1..16) */
    int32_t R;                  /* replicas per job (1..16) */
    int32_t alpha, tenure, aspiration;   /* Tabu (qb_tabu) */
    int32_t W1, W2, W3;         /* Alg. 4 weights as integers (Table 1: 2, 2, 1) */
    int32_t flags;              /* QB_RUN_* */
    const uint16_t *mlp_W_d;    /* device BF16 [4801] MLP parameters (QB_RUN_LEARNED; borrowed) */
    const float *scales_h;      /* host float [7] feature scales (qb_features); needed when learned or tracing */
    int64_t trace_capacity;     /* rows of the improvement-trace buffers; 0 = no traces */
    int32_t max_iters;          /* iterations with their own r_t and E_best trace entry (later ones reuse the last r_t) */
    int32_t rankk_variant;      /* qb_rankk variant (0 = automatic) */
    int32_t anneal_rw;          /* sparse problems: qb_anneal_ell replicas per workgroup (0 = automatic) */
} qb_run_cfg;
typedef struct {
    uint8_t *X;  int32_t *H;  int64_t *E;          /* [z][n], [z][n], [z] */
    uint8_t *xbest; int64_t *ebest;                /* [n], [1] */
    int64_t *ebest_trace;                          /* [max_iters]: E_best after iteration t */
    int32_t *T, *LF, *G;                           /* [z][n] flips, last flips, last gains */
    int64_t *K; int32_t *order;                    /* [z][n] keys and their order */
    int8_t *dX;                                    /* [z][n] */
    void *tiles;                                   /* qb_batch_info.tile_elems elements (int8 when the
                                                      problem is int8_ok, else int16), or total * ell_width
                                                      uint32 words on a sparse problem; 16-byte aligned */
    int32_t *F0; uint8_t *y0;                      /* [total] */
    uint8_t *Y; int64_t *e;                        /* [total * R], [J * R] */
    uint16_t *F;                                   /* [z][n][8] features (learned or tracing), 16-byte aligned */
    int64_t *KL; int32_t *orderL;                  /* [z][n] MLP keys and their order (learned) */
    uint16_t *trace_F; uint8_t *trace_L;           /* [trace_capacity][8], [trace_capacity] */
} qb_state_buffers;
/* Validates cfg (QB_E_ARG, QB_E_CAPACITY as qb_batch_create, qb_tabu and
 * qb_anneal state them; QB_E_RANGE when the run's instance numbers could
 * reach 2^28 within max_iters), builds the sub-QUBO batch and the
 * initial-pass batch, copies the tables, r_t for t < max_iters and the
 * scales, and allocates what bufs_h does not give.  Synchronises `stream`. */
qb_status qb_state_create(qb_state *out, qb_problem P, const qb_run_cfg *cfg, const qb_state_buffers *bufs_h,
                          void *stream);
void qb_state_destroy(qb_state S);
/* The device buffers in use (borrowed or owned) and the sub-QUBO batch. */
qb_status qb_state_get_buffers(qb_state S, qb_state_buffers *out_h);
qb_batch qb_state_batch(qb_state S);
/* Start of Alg. 2: Generate_Initial_Solution_Set (qb_init_solutions),
 * field, energy, E_best reset and best, then Call_IM_Solution_Set in
 * contiguous blocks of init_m (one after another, each seeing the previous
 * blocks' results, or all at once with QB_RUN_INIT_JACOBI); the iteration
 * record is set to t = 0 and the instance number that follows the pass. */
qb_status qb_state_init(qb_state S, void *stream);
/* `iters` outer iterations.  graph != 0: the first call captures one
 * iteration into a HIP graph (on a stream of the state's own) and every
 * iteration replays it on `stream`; graph == 0: the launches are enqueued
 * directly (such a call may itself be captured).  patience > 0 stops after
 * `patience` consecutive iterations without a lower E_best (the stall
 * criterion of the termination remark; E_best is then read after every
 * iteration, which synchronises `stream`).  *ran_h (optional) receives the
 * number of iterations run. */
qb_status qb_iterate(qb_state S, int32_t iters, int32_t graph, int32_t patience, int32_t *ran_h, void *stream);
/* The state's iteration number t and annealer instance base (synchronises
 * `stream`), and a rewind to iteration t (instance base as a run that went
 * straight from qb_state_init to t; trace rows kept) -- a kernel, so it may
 * be captured. */
qb_status qb_state_get_iteration(qb_state S, int32_t *t_h, uint32_t *inst_h, int64_t *trace_rows_h, void *stream);
qb_status qb_state_set_iteration(qb_state S, int32_t t, void *stream);
/* Write-back of the state's last annealing (Alg. 3: the best finished
 * replica of every job into X, the changes into dX), then the rank-k field
 * update, energy and best: the apply step of one iteration, for callers
 * that run the stages themselves. */
qb_status qb_apply(qb_state S, void *stream);
/* Kernel variants of later iterations (result-invariant: qb_rankk's variant,
 * qb_anneal_ell's replicas per workgroup, 0 = automatic); a captured
 * iteration is captured again. */
qb_status qb_state_set_variants(qb_state S, int32_t rankk_variant, int32_t anneal_rw);
/* Stage timing of iterations run with graph == 0: with timing on, each such
 * iteration records events at its stage boundaries, and qb_state_stage_ms
 * (synchronises `stream`) returns the last one's milliseconds for Tabu and
 * best, keys and selection, extraction, annealing, write-back with its
 * field update, and mutation with its field update (ms_h: float [6]). */
qb_status qb_state_enable_timing(qb_state S, int32_t on);
qb_status qb_state_stage_ms(qb_state S, float *ms_h, void *stream);
/* qb_check of the problem and qb_batch_check of the state's batches. */
qb_status qb_state_check(qb_state S, void *stream);

#ifdef __cplusplus
}
#endif
#endif
