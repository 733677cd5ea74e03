// Control-parameter keys (Alg. 4), rank order, plain selection (the
// selection step of Alg. 3), the job batch handle, and mutation (end of the heuristic section).
#include <math.h>

#include <algorithm>
#include <numeric>

#include "qb_internal.h"

#include <atomic>

namespace {

// c_j = sum_p X[p][j] (the column count behind gamma)
__global__ void k_colcount(const uint8_t *__restrict__ X, int n, int z, int32_t *__restrict__ cnt)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int32_t c = 0;
    // independent loads: unrolled so that many are in flight
#pragma unroll 16
    for (int p = 0; p < z; ++p) c += X[(int64_t)p * n + j];
    cnt[j] = c;
}

__global__ void __launch_bounds__(256) k_keys(int n, int z, const int64_t *__restrict__ eta,
                                              int64_t eta_max, const int32_t *__restrict__ cnt,
                                              const int32_t *__restrict__ T, int W1, int W2, int W3,
                                              int t_bound, int64_t *__restrict__ K,
                                              int32_t *__restrict__ status)
{
    __shared__ int32_t part[4];
    const int p = blockIdx.x;
    const int32_t *Tp_row = T + (int64_t)p * n;
    int32_t tm = 0;
    bool bad = false;
    for (int j = threadIdx.x; j < n; j += 256) {
        const int32_t t = Tp_row[j];
        bad |= t < 0 || t > t_bound;
        tm = max(tm, t);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) tm = max(tm, __shfl_xor(tm, o, 64));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = tm;
    if (bad) atomicOr(status, QB_FLAG_RANGE);
    __syncthreads();
    const int64_t Tp = max(max(max(part[0], part[1]), max(part[2], part[3])), 1);
    for (int j = threadIdx.x; j < n; j += 256) {
        const int32_t dev = abs(2 * cnt[j] - z);
        const int64_t g = (int64_t)z - dev;
        const int64_t dl = Tp - Tp_row[j];
        K[(int64_t)p * n + j] = (int64_t)W1 * eta[j] * z * Tp + (int64_t)W2 * g * eta_max * Tp -
                                (int64_t)W3 * dl * eta_max * z;
    }
}

// Random keys of the ablation without control parameters: one Philox word
// per (solution, variable), stream tag 4 in counter word 3.
__global__ void k_random_keys(int n, int t, const qb_iter *__restrict__ it, uint32_t k0, uint32_t k1,
                              int64_t *__restrict__ K)
{
    if (it) t = it->t;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;   // group of 4 variables
    const int p = blockIdx.y;
    if (4 * g >= n) return;
    const uint4 o = qb_philox(make_uint4((uint32_t)g, (uint32_t)t, (uint32_t)p, 4u << 28), k0, k1);
    int64_t *row = K + (int64_t)p * n;
#pragma unroll
    for (int w = 0; w < 4; ++w)
        if (4 * g + w < n) row[4 * g + w] = (int64_t)qb_word(o, w);
}

// Bitonic sort of (K desc, index asc) packed into one 64-bit key per element.
__global__ void __launch_bounds__(1024) k_rank(int n, int npad, const int64_t *__restrict__ K,
                                               int32_t *__restrict__ order)
{
    extern __shared__ uint64_t sk[];
    const int p = blockIdx.x;
    const int64_t *Kp = K + (int64_t)p * n;
    constexpr int64_t lim = (int64_t(1) << 47) - 1;
    for (int i = threadIdx.x; i < npad; i += 1024) {
        // keys are within +-lim by construction; the clamp only keeps the
        // index bits intact if a caller breaks that contract
        const int64_t k = min(max(i < n ? Kp[i] : 0, -lim), lim);
        sk[i] = i < n ? (((uint64_t)(lim - k) << 16) | (uint64_t)i) : ~0ull;
    }
    __syncthreads();
    for (int k = 2; k <= npad; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            for (int i = threadIdx.x; i < (npad >> 1); i += 1024) {
                const int lo = ((i & ~(jj - 1)) << 1) | (i & (jj - 1));
                const int hi = lo + jj;
                const bool up = (lo & k) == 0;
                const uint64_t a = sk[lo], b = sk[hi];
                if ((a > b) == up) {
                    sk[lo] = b;
                    sk[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    for (int r = threadIdx.x; r < n; r += 1024) order[(int64_t)p * n + r] = (int32_t)(sk[r] & 0xffffu);
}

// Larger n: an ascending-only bitonic network (each merge opens with the
// mirrored comparison, so every comparator puts the smaller key first and
// the virtual positions >= n act as +infinity that no comparator moves) over
// the indices held in order[p] itself; keys are rebuilt from K when needed.
// Strides below the LDS chunk run in LDS on whole chunks, longer strides on
// the indices in global memory (one workgroup per solution, so a barrier
// orders them).
constexpr int RANK_CHUNK = 16384;

__device__ __forceinline__ uint64_t rank_key(const int64_t *__restrict__ Kp, int j)
{
    constexpr int64_t lim = (int64_t(1) << 47) - 1;
    const int64_t k = min(max(Kp[j], -lim), lim);
    return ((uint64_t)(lim - k) << 16) | (uint64_t)j;
}

__device__ __forceinline__ void bitonic_positions(int i, int k, int jj, bool flip, int &lo, int &hi)
{
    if (flip) {
        const int half = k >> 1, blk = i / half, w = i - blk * half;
        lo = blk * k + w;
        hi = blk * k + k - 1 - w;
    } else {
        lo = ((i & ~(jj - 1)) << 1) | (i & (jj - 1));
        hi = lo + jj;
    }
}

// In-LDS stages of one merge of size k on a chunk: the mirrored step (when
// k <= chunk) then the half-cleaners of stride jj0, jj0/2, ..., 1.
__device__ __forceinline__ void lds_merge(uint64_t *sk, int k, bool with_flip, int jj0)
{
    constexpr int C = RANK_CHUNK;
    if (with_flip) {
        for (int i = threadIdx.x; i < C / 2; i += 1024) {
            int lo, hi;
            bitonic_positions(i, k, 0, true, lo, hi);
            const uint64_t a = sk[lo], b = sk[hi];
            if (a > b) {
                sk[lo] = b;
                sk[hi] = a;
            }
        }
        __syncthreads();
    }
    for (int jj = jj0; jj > 0; jj >>= 1) {
        for (int i = threadIdx.x; i < C / 2; i += 1024) {
            int lo, hi;
            bitonic_positions(i, 0, jj, false, lo, hi);
            const uint64_t a = sk[lo], b = sk[hi];
            if (a > b) {
                sk[lo] = b;
                sk[hi] = a;
            }
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(1024) k_rank_big(int n, int npad, const int64_t *__restrict__ K,
                                                   int32_t *__restrict__ order)
{
    constexpr int C = RANK_CHUNK;
    extern __shared__ uint64_t sk[];
    const int p = blockIdx.x;
    const int64_t *Kp = K + (int64_t)p * n;
    int32_t *op = order + (int64_t)p * n;
    const int nchunk = npad / C;
    // every chunk sorted ascending on its own
    for (int c = 0; c < nchunk; ++c) {
        for (int r = threadIdx.x; r < C; r += 1024) {
            const int g = c * C + r;
            sk[r] = g < n ? rank_key(Kp, g) : ~0ull;
        }
        __syncthreads();
        for (int k = 2; k <= C; k <<= 1) lds_merge(sk, k, true, k >> 2);
        for (int r = threadIdx.x; r < C; r += 1024) {
            const int g = c * C + r;
            if (g < n) op[g] = (int32_t)(sk[r] & 0xffffu);
        }
        __syncthreads();
    }
    // merges longer than a chunk
    for (int k = 2 * C; k <= npad; k <<= 1) {
        // the mirrored step (jj == k), then the half-cleaners of stride >= C
        for (int jj = k; jj >= C; jj = jj == k ? k >> 2 : jj >> 1) {
            const bool flip = jj == k;
            for (int i = threadIdx.x; i < npad / 2; i += 1024) {
                int lo, hi;
                bitonic_positions(i, k, flip ? 0 : jj, flip, lo, hi);
                if (hi < n) {
                    const int a = op[lo], b = op[hi];
                    if (rank_key(Kp, a) > rank_key(Kp, b)) {
                        op[lo] = b;
                        op[hi] = a;
                    }
                }
            }
            __syncthreads();
        }
        for (int c = 0; c < nchunk; ++c) {
            if (c * C >= n) break;
            for (int r = threadIdx.x; r < C; r += 1024) {
                const int g = c * C + r;
                sk[r] = g < n ? rank_key(Kp, op[g]) : ~0ull;
            }
            __syncthreads();
            lds_merge(sk, 0, false, C >> 1);
            for (int r = threadIdx.x; r < C; r += 1024) {
                const int g = c * C + r;
                if (g < n) op[g] = (int32_t)(sk[r] & 0xffffu);
            }
            __syncthreads();
        }
    }
}

// Job q: ranks [rank0, rank0+m) of its solution, sorted ascending.
__global__ void __launch_bounds__(1024) k_select(int n, const int32_t *__restrict__ sol,
                                                 const int32_t *__restrict__ off,
                                                 const int32_t *__restrict__ rank0,
                                                 const int32_t *__restrict__ order,
                                                 int32_t *__restrict__ idx)
{
    __shared__ int32_t v[1024];
    const int q = blockIdx.x;
    const int base = off[q], m = off[q + 1] - base, p = sol[q], r0 = rank0[q];
    int mpad = 1;
    while (mpad < m) mpad <<= 1;
    for (int t = threadIdx.x; t < mpad; t += 1024)
        v[t] = t < m ? order[(int64_t)p * n + r0 + t] : 0x7fffffff;
    __syncthreads();
    for (int k = 2; k <= mpad; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            for (int i = threadIdx.x; i < (mpad >> 1); i += 1024) {
                const int lo = ((i & ~(jj - 1)) << 1) | (i & (jj - 1));
                const int hi = lo + jj;
                const bool up = (lo & k) == 0;
                const int32_t a = v[lo], b = v[hi];
                if ((a > b) == up) {
                    v[lo] = b;
                    v[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < m; t += 1024) idx[base + t] = v[t];
}

// floor(a * 2^32 / b) for 0 <= a < b < 2^62 (restoring division).
__device__ __forceinline__ uint64_t frac32(uint64_t a, uint64_t b)
{
    uint64_t r = a, q = 0;
    for (int i = 0; i < 32; ++i) {
        r <<= 1;
        q <<= 1;
        if (r >= b) {
            r -= b;
            q |= 1;
        }
    }
    return q;
}

__global__ void __launch_bounds__(1024) k_mutate(int n, const int32_t *__restrict__ sol_begin,
                                                 const int32_t *__restrict__ off,
                                                 const int32_t *__restrict__ idx,
                                                 const int64_t *__restrict__ K,
                                                 const int32_t *__restrict__ order, double rate, int t,
                                                 const qb_iter *__restrict__ it,
                                                 const double *__restrict__ rate_tab, int ntab,
                                                 uint32_t k0, uint32_t k1, uint8_t *__restrict__ X,
                                                 int8_t *__restrict__ dX, int32_t *__restrict__ kcount)
{
    if (it) {
        t = it->t;
        rate = rate_tab[t < ntab ? t : ntab - 1];
    }
    __shared__ uint32_t inU[2048];
    __shared__ int wsum[16];
    const int p = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (int w = tid; w < 2048; w += 1024) inU[w] = 0;
    __syncthreads();
    const int qa = sol_begin[p], qb = sol_begin[p + 1];
    const int ua = off[qa], ub = off[qb];
    for (int a = ua + tid; a < ub; a += 1024) {
        const int j = idx[a];
        atomicOr(&inU[j >> 5], 1u << (j & 31));
    }
    __syncthreads();
    const int nc = n - (ub - ua);
    int k = (int)floor((double)nc * rate);
    if (k > nc) k = nc;
    if (k < 0) k = 0;
    if (kcount && tid == 0) kcount[p] = k;
    if (k == 0) return;
    const int64_t *Kp = K + (int64_t)p * n;
    const int32_t *op = order + (int64_t)p * n;
    const int64_t khi = Kp[op[0]], klo = Kp[op[n - 1]];
    const uint64_t den = (uint64_t)(khi - klo);
    int found = 0;
    for (int r0 = 0; r0 < n && found < k; r0 += 1024) {
        const int r = r0 + tid;
        int j = -1;
        bool c = false;
        if (r < n) {
            j = op[r];
            c = !((inU[j >> 5] >> (j & 31)) & 1u);
        }
        const uint64_t bal = __ballot(c);
        const int before = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[wid] = __popcll(bal);
        __syncthreads();
        int woff = 0, tot = 0;
        for (int w = 0; w < 16; ++w) {
            woff += w < wid ? wsum[w] : 0;
            tot += wsum[w];
        }
        const int crank = found + woff + before;
        if (c && crank < k) {
            uint64_t P;
            if (den == 0) {
                P = 1ull << 31;
            } else {
                const uint64_t a = (uint64_t)(Kp[j] - klo);
                P = a >= den ? 0xffffffffull : frac32(a, den);
            }
            const uint4 o = qb_philox(make_uint4((uint32_t)(j >> 2), (uint32_t)t, (uint32_t)p, 2u << 28), k0, k1);
            const uint32_t u = qb_word(o, j & 3);
            if ((uint64_t)u < P) {
                const int64_t at = (int64_t)p * n + j;
                const uint8_t xo = X[at];
                X[at] = xo ^ 1;
                dX[at] = xo ? -1 : 1;
            }
        }
        found += tot;
        __syncthreads();
    }
}

}  // namespace

qb_status qb_column_counts(qb_problem P, int z, const uint8_t *X, void *stream)
{
    k_colcount<<<(P->n + 255) / 256, 256, 0, qb_stream(stream)>>>(X, P->n, z, P->colcnt);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

extern "C" qb_status qb_keys(qb_problem P, int32_t z, const uint8_t *X_d, const int32_t *T_d,
                            int32_t W1, int32_t W2, int32_t W3, int32_t t_bound, int64_t *K_d,
                            void *stream)
{
    if (!P || z < 1 || !X_d || !T_d || !K_d || W1 < 0 || W2 < 0 || W3 < 0 || t_bound < 0)
        return QB_E_ARG;
    const double bound = (double)(W1 + W2 + W3) * (double)P->eta_max * (double)z *
                         (double)std::max(t_bound, 1) * 2.0;
    if (bound >= 140737488355328.0) return QB_E_RANGE;   // 2^47
    hipStream_t s = qb_stream(stream);
    qb_status rc = qb_column_counts(P, z, X_d, stream);
    if (rc != QB_OK) return rc;
    k_keys<<<z, 256, 0, s>>>(P->n, z, P->eta, P->eta_max, P->colcnt, T_d, W1, W2, W3, t_bound, K_d,
                             P->status);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

qb_status qb_random_keys_x(int32_t n, int32_t z, int32_t t, const qb_iter *it, uint64_t seed, int64_t *K_d,
                           void *stream)
{
    if (n < 1 || z < 1 || z > 65535 || t < 0 || !K_d) return QB_E_ARG;
    dim3 grid(((n + 3) / 4 + 255) / 256, z);
    k_random_keys<<<grid, 256, 0, qb_stream(stream)>>>(n, t, it, (uint32_t)seed, (uint32_t)(seed >> 32), K_d);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

extern "C" qb_status qb_random_keys(int32_t n, int32_t z, int32_t t, uint64_t seed, int64_t *K_d, void *stream)
{
    return qb_random_keys_x(n, z, t, nullptr, seed, K_d, stream);
}

extern "C" qb_status qb_rank(int32_t n, int32_t z, const int64_t *K_d, int32_t *order_d, void *stream)
{
    if (n < 1 || n > 65535 || z < 1 || !K_d || !order_d) return QB_E_ARG;
    int npad = 1;
    while (npad < n) npad <<= 1;
    npad = std::max(npad, 2);
    if (n > RANK_CHUNK) {
        static std::atomic<bool> big_attr_set{false};
        if (!big_attr_set.load(std::memory_order_acquire)) {
            QB_TRY_HIP(hipFuncSetAttribute((const void *)k_rank_big, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           RANK_CHUNK * (int)sizeof(uint64_t)));
            big_attr_set.store(true, std::memory_order_release);
        }
        k_rank_big<<<z, 1024, RANK_CHUNK * sizeof(uint64_t), qb_stream(stream)>>>(n, npad, K_d, order_d);
        QB_LAUNCH_CHECK();
        return QB_OK;
    }
    const size_t lds = sizeof(uint64_t) * npad;
    static std::atomic<bool> attr_set{false};
    if (!attr_set.load(std::memory_order_acquire)) {
        QB_TRY_HIP(hipFuncSetAttribute((const void *)k_rank, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       16384 * (int)sizeof(uint64_t)));
        attr_set.store(true, std::memory_order_release);
    }
    k_rank<<<z, 1024, lds, qb_stream(stream)>>>(n, npad, K_d, order_d);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

// ------------------------------------------------------------------ batch handle
extern "C" void qb_batch_destroy(qb_batch b)
{
    if (!b) return;
    for (void *ptr : {(void *)b->sol_d, (void *)b->off_d, (void *)b->rank0_d, (void *)b->idx_d,
                      (void *)b->sol_begin_d, (void *)b->tile_off_d, (void *)b->lpt_d, (void *)b->status_d,
                      (void *)b->dboff_d, (void *)b->iord_d, (void *)b->queue_d})
        if (ptr) (void)hipFree(ptr);
    for (int c = 0; c < QB_NCLASS; ++c) {
        if (b->side[c]) (void)hipStreamDestroy(b->side[c]);
        if (b->ev_join[c]) (void)hipEventDestroy(b->ev_join[c]);
    }
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    delete b;
}

extern "C" qb_status qb_batch_create(qb_batch *out, int32_t n, int32_t z, int32_t J,
                                    const int32_t *sol_h, const int32_t *size_h,
                                    const int32_t *rank0_h)
{
    if (!out || n < 1 || n > 65535 || z < 1 || J < 0 || (J > 0 && (!sol_h || !size_h))) return QB_E_ARG;
    *out = nullptr;
    std::vector<int64_t> per_sol(z, 0);
    for (int q = 0; q < J; ++q) {
        if (sol_h[q] < 0 || sol_h[q] >= z) return QB_E_ARG;
        if (q && sol_h[q] < sol_h[q - 1]) return QB_E_ARG;
        if (size_h[q] < 1 || size_h[q] > 1024) return QB_E_CAPACITY;
        per_sol[sol_h[q]] += size_h[q];
    }
    for (int p = 0; p < z; ++p)
        if (per_sol[p] > n) return QB_E_ARG;
    qb_batch b = new qb_batch_s();
    b->n = n;
    b->z = z;
    b->J = J;
    b->sol_h.assign(sol_h, sol_h + J);
    b->size_h.assign(size_h, size_h + J);
    b->off_h.assign(J + 1, 0);
    for (int q = 0; q < J; ++q) b->off_h[q + 1] = b->off_h[q] + size_h[q];
    b->total = b->off_h[J];
    b->m_max = J ? *std::max_element(size_h, size_h + J) : 0;
    b->rank0_h.assign(J, 0);
    {
        int cur = -1, r = 0;
        for (int q = 0; q < J; ++q) {
            if (sol_h[q] != cur) { cur = sol_h[q]; r = 0; }
            b->rank0_h[q] = rank0_h ? rank0_h[q] : r;
            if (b->rank0_h[q] < 0 || b->rank0_h[q] + size_h[q] > n) { delete b; return QB_E_ARG; }
            r += size_h[q];
        }
    }
    std::vector<int64_t> toff(J);
    int64_t acc = 0;
    for (int q = 0; q < J; ++q) {
        const int64_t mp = 64 * qb_tile_ms(size_h[q]);
        toff[q] = acc;
        acc += mp * mp;
    }
    b->tile_elems = acc;
    // diagonal 64 x 64 blocks of the sparse tiles: qb_tile_ms(m) per job
    std::vector<int32_t> dbo(J);
    int64_t nb = 0;
    for (int q = 0; q < J; ++q) {
        dbo[q] = (int32_t)nb;
        nb += qb_tile_ms(size_h[q]);
    }
    b->dblk_words = nb * 1024;
    std::vector<int32_t> sb(z + 1, J);
    for (int q = J - 1; q >= 0; --q) sb[sol_h[q]] = q;
    for (int p = z - 1; p >= 0; --p)
        if (sb[p] == J || (p + 1 <= z && sb[p] > sb[p + 1])) sb[p] = sb[p + 1];
    // class order: MS descending, within a class size descending, then job index
    std::vector<int32_t> lpt(J);
    std::iota(lpt.begin(), lpt.end(), 0);
    auto cls = [&](int q) { return qb_class_of_ms((size_h[q] + 63) / 64); };
    std::stable_sort(lpt.begin(), lpt.end(), [&](int a, int c) {
        if (cls(a) != cls(c)) return cls(a) < cls(c);
        return size_h[a] > size_h[c];
    });
    // the same classes in job index order (the queue order without LPT)
    std::vector<int32_t> iord(J);
    std::iota(iord.begin(), iord.end(), 0);
    std::stable_sort(iord.begin(), iord.end(), [&](int a, int c) { return cls(a) < cls(c); });
    for (int c = 0; c < QB_NCLASS; ++c) { b->cls_begin[c] = J; b->cls_end[c] = J; }
    for (int i = J - 1; i >= 0; --i) b->cls_begin[cls(lpt[i])] = i;
    for (int i = 0; i < J; ++i) b->cls_end[cls(lpt[i])] = i + 1;
    for (int c = 0; c < QB_NCLASS; ++c)
        if (b->cls_end[c] <= b->cls_begin[c]) b->cls_begin[c] = b->cls_end[c] = 0;

    qb_status rc = QB_OK;
    auto up = [&](void **dst, const void *src, size_t bytes) {
        if (hipMalloc(dst, std::max<size_t>(bytes, 16)) != hipSuccess) return false;
        if (hipMemset(*dst, 0, std::max<size_t>(bytes, 16)) != hipSuccess) return false;
        return bytes == 0 || hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    if (!up((void **)&b->sol_d, b->sol_h.data(), sizeof(int32_t) * J) ||
        !up((void **)&b->off_d, b->off_h.data(), sizeof(int32_t) * (J + 1)) ||
        !up((void **)&b->rank0_d, b->rank0_h.data(), sizeof(int32_t) * J) ||
        !up((void **)&b->sol_begin_d, sb.data(), sizeof(int32_t) * (z + 1)) ||
        !up((void **)&b->tile_off_d, toff.data(), sizeof(int64_t) * J) ||
        !up((void **)&b->lpt_d, lpt.data(), sizeof(int32_t) * J) ||
        !up((void **)&b->status_d, nullptr, 0) ||
        !up((void **)&b->dboff_d, dbo.data(), sizeof(int32_t) * J) ||
        !up((void **)&b->iord_d, iord.data(), sizeof(int32_t) * J) ||
        !up((void **)&b->queue_d, nullptr, 0) ||
        hipMalloc((void **)&b->idx_d, sizeof(int32_t) * std::max(b->total, 4)) != hipSuccess ||
        hipMemset(b->idx_d, 0, sizeof(int32_t) * std::max(b->total, 4)) != hipSuccess)
        rc = QB_E_HIP;
    if (rc == QB_OK) {
        if (hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess) rc = QB_E_HIP;
        // side streams only for the size classes after the first one present
        // (the first runs on the caller's stream): fewer streams share the
        // process's hardware queues, so the classes really run concurrently
        bool first = true;
        for (int c = 0; c < QB_NCLASS && rc == QB_OK; ++c) {
            if (b->cls_end[c] <= b->cls_begin[c]) continue;
            if (first) {
                first = false;
                continue;
            }
            if (hipStreamCreateWithFlags(&b->side[c], hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&b->ev_join[c], hipEventDisableTiming) != hipSuccess)
                rc = QB_E_HIP;
        }
    }
    if (rc != QB_OK) {
        qb_set_hip_error(hipGetLastError());
        qb_batch_destroy(b);
        return rc;
    }
    *out = b;
    return QB_OK;
}

extern "C" qb_status qb_batch_get_info(qb_batch b, qb_batch_info *info)
{
    if (!b || !info) return QB_E_ARG;
    info->J = b->J;
    info->total = b->total;
    info->m_max = b->m_max;
    info->tile_elems = b->tile_elems;
    info->sol_d = b->sol_d;
    info->off_d = b->off_d;
    info->idx_d = b->idx_d;
    info->dblk_words = b->dblk_words;
    return QB_OK;
}

extern "C" qb_status qb_batch_set_anneal_plan(qb_batch b, const qb_anneal_plan *plan)
{
    if (!b || !plan || plan->sleep_after < 0 ||
        (plan->depth != 8 && plan->depth != 16 && plan->depth != 32))
        return QB_E_ARG;
    for (int c = 0; c < QB_NCLASS; ++c)
        if (plan->kernel[c] < QB_ANNEAL_AUTO || plan->kernel[c] > QB_ANNEAL_MULTI_WAVE_GLOBAL) return QB_E_ARG;
    if ((plan->persistent & ~1) || (plan->lpt & ~1) || plan->wgs_per_cu < 1 || plan->wgs_per_cu > 16)
        return QB_E_ARG;
    b->plan = *plan;
    return QB_OK;
}

extern "C" qb_status qb_batch_get_anneal_plan(qb_batch b, qb_anneal_plan *plan)
{
    if (!b || !plan) return QB_E_ARG;
    *plan = b->plan;
    return QB_OK;
}

extern "C" qb_status qb_batch_count_accepts(qb_batch b, int32_t *acnt_d)
{
    if (!b) return QB_E_ARG;
    b->acnt_d = acnt_d;
    return QB_OK;
}

extern "C" qb_status qb_batch_check(qb_batch b, void *stream)
{
    if (!b) return QB_E_ARG;
    hipStream_t s = qb_stream(stream);
    int32_t st = 0;
    QB_TRY_HIP(hipMemcpyAsync(&st, b->status_d, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    QB_TRY_HIP(hipStreamSynchronize(s));
    if (st == 0) return QB_OK;
    const int32_t zero = 0;
    QB_TRY_HIP(hipMemcpyAsync(b->status_d, &zero, sizeof(int32_t), hipMemcpyHostToDevice, s));
    QB_TRY_HIP(hipStreamSynchronize(s));
    return QB_E_STATE;
}

extern "C" qb_status qb_batch_set_idx(qb_batch b, const int32_t *idx_h, void *stream)
{
    if (!b || !idx_h) return QB_E_ARG;
    std::vector<int32_t> owner(b->n, -1);
    for (int q = 0; q < b->J; ++q) {
        const int p = b->sol_h[q];
        for (int a = b->off_h[q]; a < b->off_h[q + 1]; ++a) {
            const int j = idx_h[a];
            if (j < 0 || j >= b->n) return QB_E_ARG;
            if (a > b->off_h[q] && j <= idx_h[a - 1]) return QB_E_ARG;
            if (owner[j] == p) return QB_E_OVERLAP;
            owner[j] = p;
        }
        // reset marks when the next job belongs to another solution
        if (q + 1 == b->J || b->sol_h[q + 1] != p)
            for (int q2 = q; q2 >= 0 && b->sol_h[q2] == p; --q2)
                for (int a = b->off_h[q2]; a < b->off_h[q2 + 1]; ++a) owner[idx_h[a]] = -1;
    }
    hipStream_t s = qb_stream(stream);
    QB_TRY_HIP(hipMemcpyAsync(b->idx_d, idx_h, sizeof(int32_t) * b->total, hipMemcpyHostToDevice, s));
    QB_TRY_HIP(hipStreamSynchronize(s));
    return QB_OK;
}

extern "C" qb_status qb_batch_copy_idx(qb_batch b, int32_t *idx_d, void *stream)
{
    if (!b || !idx_d) return QB_E_ARG;
    QB_TRY_HIP(hipMemcpyAsync(idx_d, b->idx_d, sizeof(int32_t) * b->total, hipMemcpyDeviceToDevice,
                              qb_stream(stream)));
    return QB_OK;
}

extern "C" qb_status qb_select(qb_batch b, const int32_t *order_d, void *stream)
{
    if (!b || !order_d) return QB_E_ARG;
    if (b->J == 0) return QB_OK;
    k_select<<<b->J, 1024, 0, qb_stream(stream)>>>(b->n, b->sol_d, b->off_d, b->rank0_d, order_d,
                                                  b->idx_d);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

qb_status qb_mutate_x(qb_batch b, const int64_t *K_d, const int32_t *order_d, double rate, int32_t t,
                      const qb_iter *it, const double *rate_tab, int32_t ntab, uint64_t seed, uint8_t *X_d,
                      int8_t *dX_d, int32_t *kcount_d, void *stream)
{
    if (!b || !K_d || !order_d || !X_d || !dX_d || !(rate >= 0.0) || t < 0) return QB_E_ARG;
    if (it && (!rate_tab || ntab < 1)) return QB_E_ARG;
    k_mutate<<<b->z, 1024, 0, qb_stream(stream)>>>(b->n, b->sol_begin_d, b->off_d, b->idx_d, K_d,
                                                  order_d, rate, t, it, rate_tab, ntab, (uint32_t)seed,
                                                  (uint32_t)(seed >> 32), X_d, dX_d, kcount_d);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

extern "C" qb_status qb_mutate(qb_batch b, const int64_t *K_d, const int32_t *order_d, double rate,
                              int32_t t, uint64_t seed, uint8_t *X_d, int8_t *dX_d, int32_t *kcount_d,
                              void *stream)
{
    return qb_mutate_x(b, K_d, order_d, rate, t, nullptr, nullptr, 0, seed, X_d, dX_d, kcount_d, stream);
}
