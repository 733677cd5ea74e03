// Internal declarations shared by the gfx950 kernels and the C-ABI wrappers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "qb.h"

// Bits of the per-problem device status word.
#define QB_FLAG_RANGE 1
#define QB_FLAG_STATE 2

struct qb_problem_s {
    int n = 0;
    const int16_t *Q = nullptr;   // borrowed, device
    int8_t *Q8 = nullptr;         // owned, device (null unless int8_ok)
    int64_t *eta = nullptr;       // owned, device [n]
    int32_t *colcnt = nullptr;    // owned, device [n] scratch for qb_keys
    int32_t *status = nullptr;    // owned, device status word
    void *Qp = nullptr;           // owned, device: Q with rows padded to ldp (int8 if int8_ok)
    void *Qt = nullptr;           // owned, device: the same rows in the dense Tabu kernel's
                                  // thread-chunk order (qb_tabu_pos), same type and pitch
    int ldp = 0;                  // row pitch of Qp and Qt in elements (qb_tabu_pitch)
    int tabu_tb = 0;              // dense Tabu workgroup size (0: n beyond its capacity)
    int tabu_ept = 0;             // dense Tabu variables per thread
    int int8_ok = 0;
    int qmax = 0;
    int64_t eta_max = 0;
    double sigma = 0.0;
    int32_t *diag = nullptr;      // owned, device [n]: Q_jj
    // sparse problems (qb_problem_create_csr): off-diagonal entries as a
    // row-major ELL, word [i*ellw + t] = (Q_ij << 16) | j for the t-th entry
    // of row i (ascending j), zero words after the last; ecnt[i] entries
    int sparse = 0;
    int ellw = 0;                 // padded to a multiple of 4
    uint32_t *ell = nullptr;      // owned, device [n * ellw]
    int32_t *ecnt = nullptr;      // owned, device [n]
    int tabu_variant = 0;         // QB_TABU_* (sparse problems)
};

// ELL word of a sparse entry and its two halves.
static inline __host__ __device__ uint32_t qb_ell_word(int32_t v, int col)
{
    return ((uint32_t)(uint16_t)(int16_t)v << 16) | (uint32_t)col;
}
static inline __host__ __device__ int qb_ell_col(uint32_t w) { return (int)(w & 0xffffu); }
static inline __host__ __device__ int32_t qb_ell_val(uint32_t w) { return (int32_t)w >> 16; }

// Threads of the dense Tabu workgroup for n variables: 1024 (sixteen waves),
// or 512 where that measured faster on MI355X.  With 1024 threads, n in
// (2048, 3072] or (4096, 5120] gives each thread 3 or 5 variables, which it
// reads in two chunks; eight waves with 5, 6 or 10 variables each then do
// the step 5-6 % faster (at n = 2500 and 5000), while elsewhere sixteen
// waves are as fast or faster (n = 1000, 4000, 6000, 7000, 8000 measured).
#define QB_TABU_THREADS 1024
static inline __host__ __device__ int qb_tabu_threads(int n)
{
    return ((n > 2048 && n <= 3072) || (n > 4096 && n <= 5120)) ? 512 : QB_TABU_THREADS;
}

// Elements per thread of the dense Tabu kernel with tb threads (the padded
// copies of Q have pitch qb_tabu_pitch(tb, EPT, element size)).  0 if n is
// too large.
static inline int qb_tabu_ept(int n, int tb)
{
    // beyond 16 elements per thread the state no longer fits 128 VGPRs
    static const int opts[] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16};
    for (int e : opts)
        if (n <= tb * e) return e;
    return 0;
}

// Elements of a thread's slot in a row of the dense Tabu kernel's copy of
// Q: when its ept elements take at most 16 bytes, the slot is rounded up to
// a power-of-two byte count, so one aligned vector load reads them (one load
// instead of 8 + 2 bytes at ept = 10, or 4 + 2 + 1 at ept = 7, with int8;
// the padding is never read into a key); beyond 16 bytes the slot is ept.
static inline __host__ __device__ int qb_tabu_slot(int ept, int esz)
{
    const int bytes = ept * esz;
    if (bytes > 16) return ept;
    int p = 1;
    while (p < bytes) p <<= 1;
    return p / esz;
}

// Row pitch of the dense Tabu copy (and of the padded copy) in elements.
static inline __host__ __device__ int qb_tabu_pitch(int tb, int ept, int esz)
{
    return tb * qb_tabu_slot(ept, esz);
}

// The dense Tabu kernel's copy of Q.  Thread t of the tb-thread workgroup
// owns the variables e * tb + t (e < ept).  Up to 16 bytes, its elements
// fill the front of its padded slot (slots in thread order).  Beyond, they
// are split into chunks of 16, 8, 4, 2 and 1 bytes (largest first, the
// largest repeated as often as it fits), and each chunk is stored for all
// threads in turn, so one naturally aligned vector load per chunk reads a
// thread's elements (one load instead of sixteen at ept = 16 with int8).
// Returns the element offset of (e, t) within the row.
static inline __host__ __device__ int qb_tabu_pos(int e, int t, int ept, int esz, int tb)
{
    if (ept * esz <= 16) return t * qb_tabu_slot(ept, esz) + e;
    int start = 0;
    for (int sz = 16 / esz; sz >= 1; sz >>= 1)
        while (ept - start >= sz) {
            if (e < start + sz) return start * tb + t * sz + (e - start);
            start += sz;
        }
    return -1;
}

// QB_OK when the sparse Tabu tree kernel can run the problem (else
// QB_E_CAPACITY or QB_E_RANGE).
qb_status qb_tabu_tree_fits(qb_problem P);

// Sparse Tabu: 1024 threads, EPT variables each (n <= 20480).
#define QB_TABU_SP_THREADS 1024
static inline int qb_tabu_sp_ept(int n)
{
    static const int opts[] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20};
    for (int e : opts)
        if (n <= QB_TABU_SP_THREADS * e) return e;
    return 0;
}

// Anneal size classes by padded width MS = mp / 64.
static constexpr int QB_NCLASS = 5;          // MS = 16, 8, 4, 2, 1
static inline int qb_class_of_ms(int ms) { return ms > 8 ? 0 : ms > 4 ? 1 : ms > 2 ? 2 : ms > 1 ? 3 : 4; }
static inline int qb_ms_of_class(int c) { return 16 >> c; }
// Padded tile width of a job of m variables: 64 * (power of two >= ceil(m/64)),
// i.e. exactly the width of the annealer class that runs it.
static inline __host__ __device__ int qb_tile_ms(int m)
{
    const int ms = (m + 63) >> 6;
    return ms > 8 ? 16 : ms > 4 ? 8 : ms > 2 ? 4 : ms > 1 ? 2 : 1;
}

struct qb_batch_s {
    int n = 0, z = 0, J = 0, total = 0, m_max = 0;
    int64_t tile_elems = 0;
    std::vector<int32_t> sol_h, off_h, size_h, rank0_h;
    int32_t *sol_d = nullptr, *off_d = nullptr, *rank0_d = nullptr, *idx_d = nullptr;
    int32_t *sol_begin_d = nullptr;   // [z+1] first job of each solution
    int64_t *tile_off_d = nullptr;    // [J]
    int32_t *lpt_d = nullptr;         // [J] jobs by class, then size descending
    int cls_begin[QB_NCLASS] = {0}, cls_end[QB_NCLASS] = {0};
    hipStream_t side[QB_NCLASS] = {nullptr};
    int32_t *status_d = nullptr;      // device status word (QB_FLAG_STATE: a job had a failed replica)
    int32_t *acnt_d = nullptr;        // optional, caller's: accepted moves per replica of the last annealing
    qb_anneal_plan plan = {16, 8, {0, 0, 0, 0, 0}, 0, 1, 1};   // annealer schedule (result-invariant)
    int32_t *iord_d = nullptr;        // [J] jobs by class, then job index (the queue order without LPT)
    int *queue_d = nullptr;           // [QB_NCLASS] job counters of the persistent annealer
    int *lq = nullptr;                // launch in progress: its class's counter (persistent) or null
    int lgrid = 0;                    // launch in progress: persistent grid (0: one workgroup per job)
    int32_t *dboff_d = nullptr;       // [J] first diagonal block of each job (sparse tiles)
    int64_t dblk_words = 0;           // words of all jobs' int8 diagonal blocks (1024 per block)
    bool dblk_valid = false;          // the last sparse extraction wrote the diagonal blocks
    hipEvent_t ev_fork = nullptr, ev_join[QB_NCLASS] = {nullptr};
};

// Per-iteration scalars of a captured outer iteration (Alg. 2), held in
// device memory so that one graph replays every iteration: kernels given a
// non-null record read t (mutation, random keys), add inst to the
// annealer's instance numbers and append traces at trn; the state's
// advance kernel moves it to the next iteration.
// Stages of one outer iteration timed by qb_state_stage_ms.
#define QB_NSTAGE 6

struct qb_iter {
    int32_t t;          // outer iteration, from 0
    uint32_t inst;      // instance number of the batch's first job
    int32_t trn;        // trace rows written
    int32_t pad;
};

// Entry points with the iteration record (nullptr: the scalars given).
qb_status qb_anneal_x(qb_batch b, const void *tile_d, int32_t int8_tile, const int32_t *F0_d, const uint8_t *y0_d,
                      int32_t nsw, int32_t B, const int32_t *thr_d, int32_t R, uint64_t seed, uint32_t inst_base,
                      const qb_iter *it, uint8_t *Y_d, int64_t *e_d, void *stream);
qb_status qb_anneal_ell_x(qb_batch b, int32_t W, const uint32_t *tile_d, const int32_t *F0_d, const uint8_t *y0_d,
                          int32_t nsw, int32_t B, const int32_t *thr_d, int32_t R, int32_t rw, uint64_t seed,
                          uint32_t inst_base, const qb_iter *it, uint8_t *Y_d, int64_t *e_d, void *stream);
// rate_tab (device, ntab entries) gives r_t for the record's t (the last
// entry beyond the table)
qb_status qb_mutate_x(qb_batch b, const int64_t *K_d, const int32_t *order_d, double rate, int32_t t,
                      const qb_iter *it, const double *rate_tab, int32_t ntab, uint64_t seed, uint8_t *X_d,
                      int8_t *dX_d, int32_t *kcount_d, void *stream);
qb_status qb_random_keys_x(int32_t n, int32_t z, int32_t t, const qb_iter *it, uint64_t seed, int64_t *K_d,
                           void *stream);
// traces appended at the record's trn when cap rows leave room (else none)
qb_status qb_trace_x(qb_batch b, int32_t R, const uint16_t *F_d, const uint8_t *Y_d, const int64_t *e_d,
                     const uint8_t *y0_d, uint16_t *outF_d, uint8_t *outL_d, const qb_iter *it, int64_t cap,
                     void *stream);

// Workgroups of an annealer launch: the persistent grid, else one per job.
static inline int qb_grid(const qb_batch_s *b, int njobs) { return b->lgrid ? b->lgrid : njobs; }
// Compute units of the current device (cached per device).
hipError_t qb_cu_count(int *out);

// Column counts c_j = sum_p X[p][j] into P->colcnt (enqueued on stream).
qb_status qb_column_counts(qb_problem P, int z, const uint8_t *X, void *stream);

// thread-local last HIP error
void qb_set_hip_error(hipError_t e);

#define QB_TRY_HIP(expr)                                   \
    do {                                                   \
        hipError_t _e = (expr);                            \
        if (_e != hipSuccess) {                            \
            qb_set_hip_error(_e);                          \
            return QB_E_HIP;                               \
        }                                                  \
    } while (0)

#define QB_LAUNCH_CHECK()                                  \
    do {                                                   \
        hipError_t _e = hipGetLastError();                 \
        if (_e != hipSuccess) {                            \
            qb_set_hip_error(_e);                          \
            return QB_E_HIP;                               \
        }                                                  \
    } while (0)

static inline hipStream_t qb_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// ------------------------------------------------------------------ device helpers
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products
// with the published multipliers, the key advanced by the published Weyl
// increments between rounds.
__device__ __forceinline__ uint4 qb_philox(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

// Replica chosen for job q (the write-back step of Alg. 3): the lowest e,
// the lowest r on ties, over the replicas that finished.  A replica whose
// bounded wait ran out reports e = INT64_MIN and is never chosen; -1 when
// no replica of the job finished.  *failed is set when any replica did not.
__device__ __forceinline__ int qb_best_replica(const int64_t *__restrict__ eq, int R, bool *failed)
{
    int rb = -1;
    bool f = false;
    for (int r = 0; r < R; ++r) {
        const int64_t v = eq[r];
        if (v == INT64_MIN) {
            f = true;
            continue;
        }
        if (rb < 0 || v < eq[rb]) rb = r;
    }
    *failed = f;
    return rb;
}

// Job slot of a workgroup's pass `pass`: without a queue, blockIdx.x on the
// first pass only; with one (the persistent annealer), the next slot of the
// atomic counter, taken by thread 0 and shared through slot_s (every thread
// of the workgroup calls this).  -1 when no job is left.
__device__ __forceinline__ int qb_next_slot(int *queue, int njobs, int pass, int *slot_s)
{
    if (!queue) return pass == 0 ? (int)blockIdx.x : -1;
    if (threadIdx.x == 0) *slot_s = atomicAdd(queue, 1);
    __syncthreads();
    const int v = *slot_s;
    __syncthreads();
    return v < njobs ? v : -1;
}

__device__ __forceinline__ uint32_t qb_word(uint4 v, int w)
{
    return w == 0 ? v.x : w == 1 ? v.y : w == 2 ? v.z : v.w;
}

// The annealers' accepted spin k: y_k is bit k of the uniform mask ym (y of
// the block's lanes at its start).  One bit test feeds the selects: first
// f = y_k ? n : p per lane (the lane's factor sigma d2 on the accepted row's
// coupling, the next step of the accept chain), then, off the chain, d2 =
// y_k ? -2 : 2 and, with YK, yk = y_k (uniform).  Written as one ALU
// sequence: the compiler otherwise builds y_k through a 64-bit shift, and,
// compare and select, all on the accept chain.
template <bool YK>
__device__ __forceinline__ void qb_accept_sign(uint64_t ym, int k, int32_t p, int32_t n, int32_t &f, int32_t &d2,
                                               int32_t &yk)
{
    if constexpr (YK) {
        asm("s_bitcmp1_b64 %[ym], %[k]\n\t"
            "s_cselect_b64 vcc, -1, 0\n\t"
            "v_cndmask_b32 %[f], %[p], %[n], vcc\n\t"
            "s_cselect_b32 %[d2], -2, 2\n\t"
            "s_cselect_b32 %[yk], 1, 0"
            : [f] "=v"(f), [d2] "=s"(d2), [yk] "=s"(yk)
            : [ym] "s"(ym), [k] "s"(k), [p] "v"(p), [n] "v"(n)
            : "vcc", "scc");
    } else {
        asm("s_bitcmp1_b64 %[ym], %[k]\n\t"
            "s_cselect_b64 vcc, -1, 0\n\t"
            "v_cndmask_b32 %[f], %[p], %[n], vcc\n\t"
            "s_cselect_b32 %[d2], -2, 2"
            : [f] "=v"(f), [d2] "=s"(d2)
            : [ym] "s"(ym), [k] "s"(k), [p] "v"(p), [n] "v"(n)
            : "vcc", "scc");
        yk = 0;
    }
}

__device__ __forceinline__ int64_t qb_wave_sum_i64(int64_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint64_t qb_wave_min_u64(uint64_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint64_t w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    return v;
}

constexpr int qb_ceil_log2(int v) { return v <= 1 ? 0 : 1 + qb_ceil_log2((v + 1) / 2); }

// Wave minimum of an unsigned value, returned uniform: DPP quad_perm
// [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror, then the four
// row results by readlane.
__device__ __forceinline__ uint32_t qb_wave_min_u32(uint32_t v)
{
    // row minimum in every lane (xor 1, xor 2, half-row mirror, row mirror),
    // then the rows meet through the gfx950 row-swap moves: no readlane and
    // no scalar round trip
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
    const auto p16 = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    v = min(v, min((uint32_t)p16[0], (uint32_t)p16[1]));
    const auto p32 = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    v = min(v, min((uint32_t)p32[0], (uint32_t)p32[1]));
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// Wave minimum, returned uniform: the row minimum in every lane (xor 1,
// xor 2, half-row mirror, row mirror), then the row broadcasts (lane 15 of
// each row into the next row, lane 31 into rows 2 and 3) leave the minimum
// of the whole wave in lane 63.  Six DPP minima and one readlane.
__device__ __forceinline__ uint32_t qb_wave_min_u32_b(uint32_t v)
{
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
    // rows outside the row mask see the identity of the minimum
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x142, 0xA, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x143, 0xC, 0xF, false));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Tabu wave winner: (biased move << 32) | (index << 1) | x_index, so the
// 64-bit minimum is the lowest move, then the lowest index.
__device__ __forceinline__ uint64_t qb_tabu_winner(uint32_t dbias, int j, uint32_t x)
{
    return ((uint64_t)dbias << 32) | ((uint64_t)(uint32_t)j << 1) | x;
}

template <int CTL>
__device__ __forceinline__ uint64_t qb_dpp_min64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTL, 0xF, 0xF, false);
    const uint64_t o = ((uint64_t)hi << 32) | lo;
    return o < v ? o : v;
}

// Tabu cross-wave winner in 32 bits: slot[w] holds, in its low word,
// (wave w's minimum key << log2 NW) | w and, in its high word,
// (lane << 1) | x.  A 32-bit DPP minimum over the first row of lanes picks
// the winning key and one readlane of that slot's high word gives its lane
// and x.  False when every slot is empty.
template <int NWV>
__device__ __forceinline__ bool qb_pick32(const uint64_t *slot, int lane, uint32_t &key, uint32_t &hi)
{
    static_assert(NWV >= 1 && NWV <= 16 && (NWV & (NWV - 1)) == 0, "a power of two, one row of 16 lanes");
    // every lane reads a slot (lanes past NWV repeat them), so no lane needs
    // a fill value and the read needs no exec mask
    const uint64_t v = slot[lane & (NWV - 1)];
    uint32_t lo = (uint32_t)v;
    lo = min(lo, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)lo, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
    lo = min(lo, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)lo, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
    // with NWV = 8 the upper half of the row repeats the lower half, so one
    // rotation by four already meets all eight slots in lane 0
    if constexpr (NWV > 4)
        lo = min(lo, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)lo, 0x124, 0xF, 0xF, false));  // row_ror 4
    if constexpr (NWV > 8)
        lo = min(lo, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)lo, 0x128, 0xF, 0xF, false));  // row_ror 8
    key = (uint32_t)__builtin_amdgcn_readfirstlane((int)lo);
    if (key == 0xFFFFFFFFu) return false;
    hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), (int)(key & (NWV - 1)));
    return true;
}

// Minimum of NW (<= 16) 64-bit values slot[0..NW), returned uniform: lane l
// of the calling wave reads slot[l] (lanes >= NW take the largest value) and
// a DPP tree inside the first row of 16 lanes (xor 1, xor 2, rotate 4,
// rotate 8) leaves the minimum in lane 0.  Must be called by a full wave.
template <int NW>
__device__ __forceinline__ uint64_t qb_min_winners(const uint64_t *slot, int lane)
{
    static_assert(NW >= 1 && NW <= 16, "one row of 16 lanes");
    uint64_t v = lane < NW ? slot[lane] : ~0ull;
    v = qb_dpp_min64<0xB1>(v);    // quad_perm [1,0,3,2]
    v = qb_dpp_min64<0x4E>(v);    // quad_perm [2,3,0,1]
    if constexpr (NW > 4) {
        v = qb_dpp_min64<0x124>(v);   // row_ror 4
        v = qb_dpp_min64<0x128>(v);   // row_ror 8
    }
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
