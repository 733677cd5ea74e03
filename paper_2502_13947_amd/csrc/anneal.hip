// Sub-QUBO extraction (eq. 4, sub-QUBO construction in Alg. 3), the batched
// Ising-machine stage and the write-back of Alg. 3 on gfx950.
//
// Annealer layout (the one-wave kernel; the multi-wave kernels below spread
// the same sweep over several waves): one replica per wave64, the R
// replicas of a job share a workgroup and its tile.  Lane L owns positions
// 64*s + L (s < MS = mp/64): their flip bases F live in VGPRs and their
// spins in a per-lane bit mask.  A sweep visits blocks of 64 positions; all
// 64 uniforms and thresholds of a block are ready before the block starts,
// the accept predicate is evaluated by every pending lane at once, and the
// lowest accepting lane k is taken (ballot + find-first-set).  After
// flipping k every lane adds 2 d T[k][own] to its F (one row read per
// accept) and only lanes after k re-evaluate: lanes before k were rejected
// with exactly the fields the sequential sweep would have shown them, so the
// result is the sequential sweep's, bit for bit, with #accepts + MS ballot
// rounds per sweep instead of m steps.
//
// Tile placement by size class: mp <= 256 (int8 or int16): whole tile in
// LDS; mp = 512 int8: the 36 upper 64x64 blocks of the symmetric tile in LDS
// (156,672 bytes, rows padded to 68 bytes so that both row and column reads
// of a block are bank-conflict free); otherwise rows stay in L2/HBM.
#include <atomic>
#include <type_traits>

#include "qb_internal.h"

namespace {

// ------------------------------------------------------------------ extract
constexpr int EXTRACT_THREADS = 512;

// The lane's MS elements of tile row a (columns 64 s + lane, s < MS, stored
// contiguously at a MP + lane MS) in one naturally aligned vector store.
template <typename TT, int MS>
__device__ __forceinline__ void store_lane_row(TT *dst, const TT (&v)[MS])
{
    constexpr int BYTES = MS * (int)sizeof(TT);
    if constexpr (BYTES >= 16) {
        uint4 w[BYTES / 16];
        __builtin_memcpy(w, v, BYTES);
#pragma unroll
        for (int t = 0; t < BYTES / 16; ++t) reinterpret_cast<uint4 *>(dst)[t] = w[t];
    } else if constexpr (BYTES == 8) {
        uint2 w;
        __builtin_memcpy(&w, v, 8);
        *reinterpret_cast<uint2 *>(dst) = w;
    } else if constexpr (BYTES == 4) {
        uint32_t w;
        __builtin_memcpy(&w, v, 4);
        *reinterpret_cast<uint32_t *>(dst) = w;
    } else if constexpr (BYTES == 2) {
        uint16_t w;
        __builtin_memcpy(&w, v, 2);
        *reinterpret_cast<uint16_t *>(dst) = w;
    } else {
        *dst = v[0];
    }
}

// Rows of one job's tile (eq. 4's T = Q[S][S] with a zero diagonal, padded
// to MP = 64 MS) and, when c is given, the linear term: wave w takes rows
// w, w + 8, ...; each lane gathers its MS columns of the row and stores them
// at once.
template <typename TT, int MS>
__device__ __forceinline__ void extract_rows(const int16_t *__restrict__ Q16, const TT *__restrict__ Qt, int n,
                                             int m, int base, int64_t xo, const int32_t *S, const uint8_t *ys,
                                             const int32_t *__restrict__ H, TT *tile, int32_t *__restrict__ c)
{
    constexpr int MP = 64 * MS, NWV = EXTRACT_THREADS / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int a = wid; a < MP; a += NWV) {
        const bool arow = a < m;
        const TT *qrow = Qt + (arow ? (int64_t)S[a] * n : 0);
        int32_t rowsum = 0;
        TT v[MS];
#pragma unroll
        for (int s = 0; s < MS; ++s) {
            const int b = 64 * s + lane;
            int32_t x = 0;
            if (arow && b < m && b != a) x = qrow[S[b]];
            v[s] = (TT)x;
            if (b < m) rowsum += x * (int32_t)ys[b];
        }
        store_lane_row<TT, MS>(tile + (int64_t)a * MP + lane * MS, v);
        if (c && arow) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) rowsum += __shfl_xor(rowsum, o, 64);
            if (lane == 0) {
                const int i = S[a];
                const int32_t qii = Q16[(int64_t)i * n + i];
                c[base + a] = qii + 2 * (H[xo + i] - qii * (int32_t)ys[a]) - 2 * rowsum;
            }
        }
    }
}

template <typename TT>
__global__ void __launch_bounds__(EXTRACT_THREADS) k_extract(const int16_t *__restrict__ Q16, const TT *__restrict__ Qt,
                                                 int n, const int32_t *__restrict__ sol,
                                                 const int32_t *__restrict__ off,
                                                 const int64_t *__restrict__ tile_off,
                                                 const int32_t *__restrict__ idx,
                                                 const uint8_t *__restrict__ X,
                                                 const int32_t *__restrict__ H, TT *__restrict__ tiles,
                                                 int32_t *__restrict__ c, int32_t *__restrict__ F0,
                                                 uint8_t *__restrict__ y0)
{
    __shared__ int32_t S[1024];
    __shared__ uint8_t ys[1024];
    const int q = blockIdx.x, tid = threadIdx.x;
    const int base = off[q], m = off[q + 1] - base, p = sol[q];
    const int64_t xo = (int64_t)p * n;
    for (int a = tid; a < m; a += EXTRACT_THREADS) {
        const int j = idx[base + a];
        S[a] = j;
        ys[a] = X[xo + j];
    }
    __syncthreads();
    for (int a = tid; a < m; a += EXTRACT_THREADS) {
        const int i = S[a];
        const int32_t qii = Q16[(int64_t)i * n + i];
        F0[base + a] = qii + 2 * (H[xo + i] - qii * (int32_t)ys[a]);
        y0[base + a] = ys[a];
    }
    TT *tile = tiles + tile_off[q];
    switch (qb_tile_ms(m)) {
    case 1: extract_rows<TT, 1>(Q16, Qt, n, m, base, xo, S, ys, H, tile, c); break;
    case 2: extract_rows<TT, 2>(Q16, Qt, n, m, base, xo, S, ys, H, tile, c); break;
    case 4: extract_rows<TT, 4>(Q16, Qt, n, m, base, xo, S, ys, H, tile, c); break;
    case 8: extract_rows<TT, 8>(Q16, Qt, n, m, base, xo, S, ys, H, tile, c); break;
    default: extract_rows<TT, 16>(Q16, Qt, n, m, base, xo, S, ys, H, tile, c); break;
    }
}

// ------------------------------------------------------------------ anneal
constexpr int SYM_STRIDE = 68;                   // bytes per row of a stored 64x64 block
constexpr int SYM_BLOCK = 64 * SYM_STRIDE;       // 4352
constexpr int SYM_BYTES = 36 * SYM_BLOCK;        // 156,672

__device__ __forceinline__ int sym_block_index(int a, int b)   // a <= b < 8
{
    return a * 8 - (a * (a - 1)) / 2 + (b - a);
}

// Sum of the accepted dE of one block (at most 64 moves).  With int8 tiles
// the problem has |Q| <= 127, so |dE| <= |F| <= 127 (2n + 1) < 2^24 and 32
// bits hold the sum; int16 tiles sum in 64 bits.
template <typename TT>
using block_esum = typename std::conditional<sizeof(TT) == 1, int32_t, int64_t>::type;

template <int MS, typename TT>
struct RowVec {
    TT v[MS];
};

// MODE 0: whole tile in LDS; MODE 1: symmetric 64x64 blocks in LDS (int8,
// MS = 8); MODE 2: rows read from global memory.
template <int MS, typename TT, int MODE>
__device__ __forceinline__ void fetch_row(const uint8_t *lds, const TT *__restrict__ gtile, int row, int lane,
                                          int32_t (&rv)[MS])
{
    constexpr int MP = 64 * MS;
    if constexpr (MODE == 1) {
        const int a = row >> 6, rr = row & 63;
#pragma unroll
        for (int s = 0; s < MS; ++s) {
            const int off = s >= a ? sym_block_index(a, s) * SYM_BLOCK + rr * SYM_STRIDE + lane
                                   : sym_block_index(s, a) * SYM_BLOCK + lane * SYM_STRIDE + rr;
            rv[s] = (int32_t)(int8_t)lds[off];
        }
    } else {
        const TT *src;
        if constexpr (MODE == 0)
            src = reinterpret_cast<const TT *>(lds) + (size_t)row * MP + lane * MS;
        else
            src = gtile + (size_t)row * MP + lane * MS;
        RowVec<MS, TT> r;
        if constexpr (MS * sizeof(TT) >= 16) {
#pragma unroll
            for (int c = 0; c < (int)(MS * sizeof(TT) / 16); ++c)
                reinterpret_cast<uint4 *>(&r)[c] = reinterpret_cast<const uint4 *>(src)[c];
        } else {
            r = *reinterpret_cast<const RowVec<MS, TT> *>(src);
        }
#pragma unroll
        for (int s = 0; s < MS; ++s) rv[s] = (int32_t)r.v[s];
    }
}

template <int MS, typename TT, int MODE>
struct AnnealLds {
    static constexpr size_t bytes = MODE == 0 ? (size_t)64 * MS * 64 * MS * sizeof(TT) : MODE == 1 ? SYM_BYTES : 16;
};

template <int MS, typename TT, int MODE>
__device__ __forceinline__ void anneal_job(int slot, const int32_t *__restrict__ jobs, const int32_t *__restrict__ off,
                                                 const int64_t *__restrict__ tile_off,
                                                 const TT *__restrict__ tiles, const int32_t *__restrict__ F0,
                                                 const uint8_t *__restrict__ y0, int nsw, int B,
                                                 const int32_t *__restrict__ thr, int R, uint32_t k0,
                                                 uint32_t k1, uint32_t inst_base, const qb_iter *__restrict__ it, uint8_t *__restrict__ Y,
                                                 int64_t *__restrict__ eout, int32_t *__restrict__ acnt)
{
    constexpr int MP = 64 * MS;
    __shared__ __align__(16) uint8_t lds[AnnealLds<MS, TT, MODE>::bytes];
    const int q = jobs[slot];
    const int base = off[q], m = off[q + 1] - base;
    const TT *gtile = tiles + tile_off[q];
    const int tid = threadIdx.x, lane = tid & 63, r = tid >> 6;

    if constexpr (MODE == 0) {
        constexpr int n16 = (int)(AnnealLds<MS, TT, MODE>::bytes / 16);
        const uint4 *src = reinterpret_cast<const uint4 *>(gtile);
        uint4 *dst = reinterpret_cast<uint4 *>(lds);
        for (int t = tid; t < n16; t += blockDim.x) dst[t] = src[t];
        __syncthreads();
    } else if constexpr (MODE == 1) {
        // row x, column chunk cc: 8 bytes = T[x][64 b + cc] for b = 0..7
        const uint64_t *src = reinterpret_cast<const uint64_t *>(gtile);
        for (int t = tid; t < MP * 64; t += blockDim.x) {
            const int x = t >> 6, cc = t & 63;
            const uint64_t w = src[t];
            const int a = x >> 6, rr = x & 63;
#pragma unroll
            for (int b = 0; b < 8; ++b)
                if (b >= a) lds[sym_block_index(a, b) * SYM_BLOCK + rr * SYM_STRIDE + cc] = (uint8_t)(w >> (8 * b));
        }
        __syncthreads();
    }

    int32_t F[MS];
    uint32_t ybits = 0;
    uint64_t active[MS];
#pragma unroll
    for (int s = 0; s < MS; ++s) {
        const int pos = 64 * s + lane;
        F[s] = pos < m ? F0[base + pos] : 0;
        if (pos < m && y0[base + pos]) ybits |= 1u << s;
        const int na = min(max(m - 64 * s, 0), 64);
        active[s] = na == 64 ? ~0ull : ((1ull << na) - 1ull);
    }
    int64_t e = 0;
    int32_t nacc = 0;
    const uint32_t tag = (1u << 28) | (inst_base + (it ? it->inst : 0u) + (uint32_t)q);
    constexpr int G = (MS + 3) / 4;
    const int sh = 32 - B;

    for (int sw = 0; sw < nsw; ++sw) {
        uint32_t u[4 * G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint4 o = qb_philox(make_uint4(((uint32_t)g << 6) | (uint32_t)lane, (uint32_t)sw, (uint32_t)r, tag), k0, k1);
            u[4 * g + 0] = o.x;
            u[4 * g + 1] = o.y;
            u[4 * g + 2] = o.z;
            u[4 * g + 3] = o.w;
        }
        const int32_t *ts = thr + ((size_t)sw << B);
        int32_t tv[MS];
#pragma unroll
        for (int s = 0; s < MS; ++s) tv[s] = ts[u[s] >> sh];
#pragma unroll
        for (int s = 0; s < MS; ++s) {
            uint64_t pend = active[s];
            block_esum<TT> eb = 0;
            int cb = 0;
            while (true) {
                const uint32_t yb = (ybits >> s) & 1u;
                const int32_t dE = yb ? -F[s] : F[s];
                const uint64_t acc = __ballot(dE <= tv[s]) & pend;
                if (acc == 0) break;
                const int k = __builtin_ctzll(acc);
                const int32_t dEk = __builtin_amdgcn_readlane(dE, k);
                const int32_t ykb = __builtin_amdgcn_readlane((int32_t)yb, k);
                eb += dEk;
                ++cb;
                const int32_t d2 = ykb ? -2 : 2;
                if (lane == k) ybits ^= 1u << s;
                int32_t rv[MS];
                fetch_row<MS, TT, MODE>(lds, gtile, 64 * s + k, lane, rv);
#pragma unroll
                for (int s2 = 0; s2 < MS; ++s2) F[s2] += d2 * rv[s2];
                pend &= ~((2ull << k) - 1ull);
            }
            e += eb;
            nacc += cb;
        }
    }

    uint8_t *Yr = Y + (size_t)base * R + (size_t)r * m;
#pragma unroll
    for (int s = 0; s < MS; ++s) {
        const int pos = 64 * s + lane;
        if (pos < m) Yr[pos] = (uint8_t)((ybits >> s) & 1u);
    }
    if (lane == 0) eout[(size_t)q * R + r] = e;
    if (acnt && lane == 0) acnt[(size_t)q * R + r] = nacc;
}
template <int MS, typename TT, int MODE>
__global__ void __launch_bounds__(1024) k_anneal(const int32_t *__restrict__ jobs, const int32_t *__restrict__ off,
                                                 const int64_t *__restrict__ tile_off,
                                                 const TT *__restrict__ tiles, const int32_t *__restrict__ F0,
                                                 const uint8_t *__restrict__ y0, int nsw, int B,
                                                 const int32_t *__restrict__ thr, int R, uint32_t k0,
                                                 uint32_t k1, uint32_t inst_base, const qb_iter *__restrict__ it, uint8_t *__restrict__ Y,
                                                 int64_t *__restrict__ eout, int32_t *__restrict__ acnt,
        int *__restrict__ queue, int njobs)
{
    __shared__ int slot_s;
    for (int pass = 0;; ++pass) {
        const int slot = qb_next_slot(queue, njobs, pass, &slot_s);
        if (slot < 0) break;
        anneal_job<MS, TT, MODE>(slot, jobs, off, tile_off, tiles, F0, y0, nsw, B, thr, R, k0, k1, inst_base, it, Y, eout, acnt);
        __syncthreads();   // the next job reuses the workgroup's LDS
    }
}


template <int MS, typename TT, int MODE>
void launch_anneal(int nblocks, int R, hipStream_t s, const int32_t *jobs, qb_batch b, const void *tiles,
                   const int32_t *F0, const uint8_t *y0, int nsw, int B, const int32_t *thr, uint64_t seed,
                   uint32_t inst_base, const qb_iter *it, uint8_t *Y, int64_t *e)
{
    k_anneal<MS, TT, MODE><<<qb_grid(b, nblocks), 64 * R, 0, s>>>(jobs, b->off_d, b->tile_off_d, (const TT *)tiles,
                                                                   F0, y0, nsw, B, thr, R, (uint32_t)seed,
                                                                   (uint32_t)(seed >> 32), inst_base, it, Y, e,
                                                                   b->acnt_d, b->lq, nblocks);
}

// ------------------------------------------------------------ anneal, waves
// The same sweep with the blocks of a replica spread over NW = min(MS, 4)
// waves (one per SIMD): wave w owns the NB = MS/NW consecutive blocks
// s = w NB .. w NB + NB - 1 -- their F in VGPRs, their spins as sign masks,
// and the diagonal 64x64 block of each packed in VGPRs -- and runs the
// accept loops of its blocks when its turn comes.  Every accept is published
// as one word in an LDS list (the list of block sequence number
// G = sw MS + s), and the other waves fold the accepted rows into their own
// F while the owner is still sweeping.  A wave starts its turn once it has
// applied every list before it, so each decision sees exactly the fields of
// the sequential sweep (integer sums do not depend on the order of the
// additions): Y and e are bit-identical to the one-wave kernel.  The owner's
// per-accept chain reads the flipped row's element in its own block from
// registers (an indexed register move), with no memory access on it.
//
// Lists: MS per replica, list G in slot G % MS, 65 words (64 accepts and an
// end mark), word = (G+1) << 8 | k << 1 | (y_k before the flip).  When the
// owner of G writes its list, every other wave has started a turn after
// G - MS and so has read list G - MS to its end: the ring never overwrites
// an unread list.  Every wait is bounded (qb_set_anneal_wait_limit polls,
// 2^24 by default); a replica whose wait runs out reports e = INT64_MIN.
constexpr int MW_SLOTS = 65;
constexpr int MW_LDS_LIMIT = 163840;
// polls of one word before a wave gives up (qb_set_anneal_wait_limit); the
// kernels take it as a constant unless it was changed from the default
constexpr int32_t MW_WAIT_DEFAULT = 1 << 24;
std::atomic<int32_t> g_wait_limit{MW_WAIT_DEFAULT};

template <int MS, typename TT, int MODE>
struct AnnealMw {
    static constexpr int NW = MS < 4 ? MS : 4;                 // waves per replica
    static constexpr int NB = MS / NW;                         // blocks per wave
    static constexpr int DW = 64 * (int)sizeof(TT) / 4;        // dwords of a packed diagonal column
    static constexpr size_t tile = MODE == 0 ? (size_t)64 * MS * 64 * MS * sizeof(TT) : SYM_BYTES;
    static constexpr size_t list_bytes = (size_t)MS * MW_SLOTS * 4;
    static constexpr int RWAVES = 16 / NW;                     // replicas of 1024 threads
    static constexpr int RLDS = (int)((MW_LDS_LIMIT - tile - 256) / list_bytes);
    static constexpr int RMAX = RWAVES < RLDS ? RWAVES : RLDS;
};

// Address of T[64 a + k][64 cb + lane] in the staged tile as
// base + k * ks + lane * ls: base and the strides depend only on the row
// block a and the column block cb, so they are formed once per list and
// block, leaving one multiply-add per element.
struct ElemAddr {
    int base, ks, ls;
};

template <int MS, typename TT, int MODE>
__device__ __forceinline__ ElemAddr elem_addr(int a, int cb)
{
    if constexpr (MODE == 1) {
        if (cb >= a) return ElemAddr{sym_block_index(a, cb) * SYM_BLOCK, SYM_STRIDE, 1};
        return ElemAddr{sym_block_index(cb, a) * SYM_BLOCK, 1, SYM_STRIDE};
    } else {
        constexpr int MP = 64 * MS;
        return ElemAddr{64 * a * MP + cb, MP, MS};
    }
}

template <typename TT, int MODE>
__device__ __forceinline__ int32_t elem_at(const uint8_t *lds, const ElemAddr &ea, int k, int lane)
{
    const int o = ea.base + k * ea.ks + lane * ea.ls;
    if constexpr (MODE == 1)
        return (int32_t)(int8_t)lds[o];
    else
        return (int32_t)reinterpret_cast<const TT *>(lds)[o];
}

// element k of a packed diagonal column (k uniform: an indexed register move)
template <typename TT, int DW>
__device__ __forceinline__ int32_t diag_at(const uint32_t (&d)[DW], int k)
{
    // v_bfe_i32 takes its offset modulo 32 (bits [4:0]): 8 k and 16 k select
    // the element within the word without a mask
    if constexpr (sizeof(TT) == 1)
        return __builtin_amdgcn_sbfe((int)d[k >> 2], (uint32_t)k * 8u, 8u);
    else
        return __builtin_amdgcn_sbfe((int)d[k >> 1], (uint32_t)k * 16u, 16u);
}

template <int MS, typename TT, int MODE, bool LIM>
__device__ __forceinline__ void anneal_mw_job(int slot, const int32_t *__restrict__ jobs, const int32_t *__restrict__ off,
                                                    const int64_t *__restrict__ tile_off,
                                                    const TT *__restrict__ tiles, const int32_t *__restrict__ F0,
                                                    const uint8_t *__restrict__ y0, int nsw, int B,
                                                    const int32_t *__restrict__ thr, int R, uint32_t k0,
                                                    uint32_t k1, uint32_t inst_base, const qb_iter *__restrict__ it, uint8_t *__restrict__ Y,
                                                    int64_t *__restrict__ eout, int32_t *__restrict__ acnt,
                                                    int wait_limit, int sleep_after)
{
    using C = AnnealMw<MS, TT, MODE>;
    constexpr int NW = C::NW, NB = C::NB, DW = C::DW, MP = 64 * MS;
    constexpr int PER = 4 / (int)sizeof(TT);
    __shared__ __align__(16) uint8_t lds[C::tile];
    __shared__ uint32_t lists[C::RMAX][MS][MW_SLOTS];
    __shared__ int64_t esum[16];
    __shared__ int32_t asum[16];
    __shared__ int32_t bad[C::RMAX];
    const int q = jobs[slot];
    const int base = off[q], m = off[q + 1] - base;
    const TT *gtile = tiles + tile_off[q];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wg = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r = wg / NW, w = wg - r * NW;
    const int s0 = w * NB;                       // first own block

    if constexpr (MODE == 0) {
        constexpr int n16 = (int)(C::tile / 16);
        const uint4 *src = reinterpret_cast<const uint4 *>(gtile);
        uint4 *dst = reinterpret_cast<uint4 *>(lds);
        for (int t = tid; t < n16; t += blockDim.x) dst[t] = src[t];
    } else {
        const uint64_t *src = reinterpret_cast<const uint64_t *>(gtile);
        for (int t = tid; t < MP * 64; t += blockDim.x) {
            const int x = t >> 6, cc = t & 63;
            const uint64_t v = src[t];
            const int a = x >> 6, rr = x & 63;
#pragma unroll
            for (int b = 0; b < 8; ++b)
                if (b >= a) lds[sym_block_index(a, b) * SYM_BLOCK + rr * SYM_STRIDE + cc] = (uint8_t)(v >> (8 * b));
        }
    }
    for (int t = tid; t < C::RMAX * MS * MW_SLOTS; t += blockDim.x) (&lists[0][0][0])[t] = 0u;
    if (tid < C::RMAX) bad[tid] = 0;
    __syncthreads();

    uint32_t(*L)[MW_SLOTS] = lists[r];
    int32_t F[NB], M[NB];      // M: 0 or -1 (= -y) for position 64 (s0 + j) + lane
    uint64_t active[NB];
    uint32_t dcol[NB][DW];     // T[64 s + k][64 s + lane] for k = 0..63, packed
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int pos = 64 * (s0 + j) + lane;
        F[j] = pos < m ? F0[base + pos] : 0;
        M[j] = (pos < m && y0[base + pos]) ? -1 : 0;
        const int na = min(max(m - 64 * (s0 + j), 0), 64);
        active[j] = na == 64 ? ~0ull : ((1ull << na) - 1ull);
        const ElemAddr ed = elem_addr<MS, TT, MODE>(s0 + j, s0 + j);
#pragma unroll
        for (int i = 0; i < DW; ++i) {
            uint32_t wv = 0;
#pragma unroll
            for (int t = 0; t < PER; ++t)
                wv |= ((uint32_t)elem_at<TT, MODE>(lds, ed, i * PER + t, lane) & (0xFFFFFFFFu >> (32 - 32 / PER)))
                      << (t * (32 / PER));
            dcol[j][i] = wv;
        }
    }
    const uint32_t tag = (1u << 28) | (inst_base + (it ? it->inst : 0u) + (uint32_t)q);
    const int sh = 32 - B;
    // thresholds of one sweep for the own blocks: they lie in one Philox
    // group (s0 >> 2), the uniform of block s being word s & 3
    auto thresholds = [&](int sw, int32_t (&tv)[NB]) {
        const uint4 o = qb_philox(make_uint4(((uint32_t)(s0 >> 2) << 6) | (uint32_t)lane, (uint32_t)sw, (uint32_t)r, tag),
                                  k0, k1);
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int sq = (s0 + j) & 3;
            const uint32_t uw = sq == 0 ? o.x : sq == 1 ? o.y : sq == 2 ? o.z : o.w;
            tv[j] = thr[((size_t)sw << B) + (uw >> sh)];
        }
    };
    // fetched one sweep ahead, right after the turn
    int32_t tvn[NB];
    thresholds(0, tvn);
    int64_t e = 0;
    int32_t nacc = 0;
    int Gc = 0;                // next list this wave has to apply
    bool ok = true;

    for (int sw = 0; sw < nsw && ok; ++sw) {
        const int G0 = sw * MS + s0;
        for (; Gc < G0; ++Gc) {
            const int sc = Gc & (MS - 1);
            if (sc >= s0 && sc < s0 + NB) continue;       // own list: applied while produced
            const uint32_t want = (uint32_t)(Gc + 1);
            const uint32_t *lst = L[sc];
            ElemAddr ea[NB];
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) ea[jj] = elem_addr<MS, TT, MODE>(sc, s0 + jj);
            int idx = 0;
            uint32_t v = (uint32_t)__builtin_amdgcn_readfirstlane(
                (int)__hip_atomic_load(&lst[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
            while (true) {
                int spins = 0;
                while ((v >> 8) != want) {
                    if (++spins > (LIM ? wait_limit : MW_WAIT_DEFAULT)) {
                        ok = false;
                        break;
                    }
                    if (spins > sleep_after) __builtin_amdgcn_s_sleep(1);
                    v = (uint32_t)__builtin_amdgcn_readfirstlane(
                        (int)__hip_atomic_load(&lst[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
                }
                if (!ok) break;
                const int k = (int)((v >> 1) & 127u);
                if (k == 64) break;                         // end of list
                const int32_t d2 = (v & 1u) ? -2 : 2;
                int32_t t[NB];
#pragma unroll
                for (int jj = 0; jj < NB; ++jj) t[jj] = elem_at<TT, MODE>(lds, ea[jj], k, lane);
                // the next word is read together with the row elements
                ++idx;
                v = (uint32_t)__builtin_amdgcn_readfirstlane(
                    (int)__hip_atomic_load(&lst[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
#pragma unroll
                for (int jj = 0; jj < NB; ++jj) F[jj] += d2 * t[jj];
            }
            if (!ok) break;
        }
        if (!ok) break;

        int32_t tv[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) tv[j] = tvn[j];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int s = s0 + j;
            const int G = G0 + j;
            uint32_t *out = L[s];
            const uint32_t gt = (uint32_t)(G + 1) << 8;
            ElemAddr ea[NB];
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) ea[jj] = elem_addr<MS, TT, MODE>(s, s0 + jj);
            uint64_t pend = active[j];
            block_esum<TT> ej = 0;
            int c = 0;
            // the turn works on dE = sigma F (sigma = 1 - 2y) itself.  A lane
            // that flips has its sigma negated, but its dE is not read again
            // in the turn (pend) and the negation commutes with the later
            // updates, so every flip is applied at the end: there F = sigma dE
            // with the sigma of the turn's start, for every lane, and y comes
            // from the scalar mask
            const int32_t M0 = M[j];
            const int32_t s2 = M0 ? -2 : 2, ns2 = -s2;    // 2 sigma
            int32_t dE = (F[j] ^ M0) - M0;
            uint64_t acc = __ballot(dE <= tv[j]) & pend;
            // y of the block's lanes at the turn's start, in scalar registers:
            // a lane accepts at most once in the turn, so an accepted lane's y
            // is still this bit
            const uint64_t ym0 = __ballot(M0 != 0);
            uint64_t amask = 0;                          // lanes accepted in the turn
            // the accepted row's elements in the wave's other blocks are read
            // after the accept's decision and added one accept later, so the
            // LDS read is not waited for on the accept chain
            int32_t pt[NB];
            int32_t pd2 = 0;
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) pt[jj] = 0;
            while (acc) {
                const int k = __builtin_ctzll(acc);
                const uint64_t bk = 1ull << k;
                ej += __builtin_amdgcn_readlane(dE, k);
                amask |= bk;
                // (the bit test of qb_accept_sign measured slower in this kernel)
                const bool mk = (ym0 & bk) != 0ull;
                const int32_t d2 = mk ? -2 : 2;                // y_k = 0: +2, y_k = 1: -2
                dE += (mk ? ns2 : s2) * diag_at<TT, DW>(dcol[j], k);
                // every lane stores the same word
                __hip_atomic_store(&out[c], gt | ((uint32_t)k << 1) | (mk ? 1u : 0u), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                ++c;
                pend &= (~0ull << k) << 1;
                acc = __ballot(dE <= tv[j]) & pend;
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int jj = 0; jj < NB; ++jj)
                    if (jj != j) {
                        F[jj] += pd2 * pt[jj];
                        pt[jj] = elem_at<TT, MODE>(lds, ea[jj], k, lane);
                    }
                pd2 = d2;
            }
#pragma unroll
            for (int jj = 0; jj < NB; ++jj)
                if (jj != j) F[jj] += pd2 * pt[jj];
            F[j] = (dE ^ M0) - M0;
            M[j] = (((ym0 ^ amask) >> lane) & 1ull) ? -1 : 0;
            __hip_atomic_store(&out[c], gt | (64u << 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            e += ej;
            nacc += c;
        }
        Gc = G0 + NB;
        if (sw + 1 < nsw) thresholds(sw + 1, tvn);
    }

    if (!ok && lane == 0) __hip_atomic_store(&bad[r], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (lane == 0) esum[wg] = e;
    if (lane == 0) asum[wg] = nacc;
    uint8_t *Yr = Y + (size_t)base * R + (size_t)r * m;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int pos = 64 * (s0 + j) + lane;
        if (pos < m) Yr[pos] = (uint8_t)(M[j] & 1);
    }
    __syncthreads();
    if (w == 0 && lane == 0) {
        int64_t t = 0;
        int32_t na = 0;
        for (int v = 0; v < NW; ++v) {
            t += esum[r * NW + v];
            na += asum[r * NW + v];
        }
        eout[(size_t)q * R + r] = bad[r] ? INT64_MIN : t;
        if (acnt) acnt[(size_t)q * R + r] = na;
    }
}
template <int MS, typename TT, int MODE, bool LIM>
__global__ void __launch_bounds__(1024) k_anneal_mw(const int32_t *__restrict__ jobs, const int32_t *__restrict__ off,
                                                    const int64_t *__restrict__ tile_off,
                                                    const TT *__restrict__ tiles, const int32_t *__restrict__ F0,
                                                    const uint8_t *__restrict__ y0, int nsw, int B,
                                                    const int32_t *__restrict__ thr, int R, uint32_t k0,
                                                    uint32_t k1, uint32_t inst_base, const qb_iter *__restrict__ it, uint8_t *__restrict__ Y,
                                                    int64_t *__restrict__ eout, int32_t *__restrict__ acnt,
                                                    int wait_limit, int sleep_after,
        int *__restrict__ queue, int njobs)
{
    __shared__ int slot_s;
    for (int pass = 0;; ++pass) {
        const int slot = qb_next_slot(queue, njobs, pass, &slot_s);
        if (slot < 0) break;
        anneal_mw_job<MS, TT, MODE, LIM>(slot, jobs, off, tile_off, tiles, F0, y0, nsw, B, thr, R, k0, k1, inst_base, it, Y, eout, acnt, wait_limit, sleep_after);
        __syncthreads();   // the next job reuses the workgroup's LDS
    }
}


template <int MS, typename TT, int MODE>
bool launch_anneal_mw(int nblocks, int R, hipStream_t s, const int32_t *jobs, qb_batch b, const void *tiles,
                      const int32_t *F0, const uint8_t *y0, int nsw, int B, const int32_t *thr, uint64_t seed,
                      uint32_t inst_base, const qb_iter *it, uint8_t *Y, int64_t *e)
{
    using C = AnnealMw<MS, TT, MODE>;
    // replicas per workgroup, and list tags G + 1 < 2^24 that cannot wrap
    if (R > C::RMAX || (int64_t)nsw * MS + 1 >= (int64_t(1) << 24)) return false;
    const int32_t lim = g_wait_limit.load(std::memory_order_relaxed);
    if (lim == MW_WAIT_DEFAULT)
        k_anneal_mw<MS, TT, MODE, false><<<qb_grid(b, nblocks), 64 * C::NW * R, 0, s>>>(
            jobs, b->off_d, b->tile_off_d, (const TT *)tiles, F0, y0, nsw, B, thr, R, (uint32_t)seed,
            (uint32_t)(seed >> 32), inst_base, it, Y, e, b->acnt_d, lim, b->plan.sleep_after, b->lq, nblocks);
    else
        k_anneal_mw<MS, TT, MODE, true><<<qb_grid(b, nblocks), 64 * C::NW * R, 0, s>>>(
            jobs, b->off_d, b->tile_off_d, (const TT *)tiles, F0, y0, nsw, B, thr, R, (uint32_t)seed,
            (uint32_t)(seed >> 32), inst_base, it, Y, e, b->acnt_d, lim, b->plan.sleep_after, b->lq, nblocks);
    return true;
}

// ------------------------------------------------ anneal, waves, rows in HBM
// The multi-wave sweep for tiles that do not fit LDS (mp = 1024 int8,
// mp = 512 int16; 16 bytes of every row per lane).  Wave w owns the NB
// consecutive blocks s0 = w NB ..; it keeps their diagonal 64x64 blocks in
// VGPRs and the off-diagonal blocks of its own NB x NB square in LDS, so
// the owner's accept loop touches no global memory.  The other waves fetch,
// for each published accept, the one dword of the accepted row that holds
// their NB column blocks (row k, bytes 16 lane + 4 w), up to P loads in
// flight per batch of list words.  Lists, ring and bounded waits as in the
// in-LDS multi-wave kernel.
template <int MS, typename TT, int PD>
struct AnnealMwG {
    static constexpr int NW = MS < 4 ? MS : 4;
    static constexpr int NB = MS / NW;
    static constexpr int DW = 64 * (int)sizeof(TT) / 4;
    static constexpr int PER = 4 / (int)sizeof(TT);
    static constexpr int OSTR = 64 * (int)sizeof(TT) + 4;      // bytes per row of a stored block
    static constexpr int OBLK = 64 * OSTR;
    static constexpr int NOFF = NB * (NB - 1) / 2;             // own off-diagonal blocks
    static constexpr int P = PD;                               // list words per consumer batch
    static constexpr int SLOTS = 65 + P - 1;
    static constexpr int LB = NB * (int)sizeof(TT);            // bytes of a row a consumer reads
    static_assert(LB == 1 || LB == 2 || LB == 4, "one load of 1, 2 or 4 bytes per consumer row");
};

// one consumer load of LB bytes, zero-extended
template <int LB>
__device__ __forceinline__ uint32_t load_lb(const uint8_t *p)
{
    if constexpr (LB == 4) return *reinterpret_cast<const uint32_t *>(p);
    else if constexpr (LB == 2) return *reinterpret_cast<const uint16_t *>(p);
    else return *p;
}

__device__ __forceinline__ int own_pair(int a, int b, int nb)   // a < b < nb
{
    return a * nb - (a * (a + 1)) / 2 + (b - a - 1);
}

template <int MS, typename TT, bool LIM, int PD>
__device__ __forceinline__ void anneal_mw_g_job(int slot, const int32_t *__restrict__ jobs,
                                                     const int32_t *__restrict__ off,
                                                     const int64_t *__restrict__ tile_off,
                                                     const TT *__restrict__ tiles, const int32_t *__restrict__ F0,
                                                     const uint8_t *__restrict__ y0, int nsw, int B,
                                                     const int32_t *__restrict__ thr, int R, uint32_t k0,
                                                     uint32_t k1, uint32_t inst_base, const qb_iter *__restrict__ it, uint8_t *__restrict__ Y,
                                                     int64_t *__restrict__ eout, int32_t *__restrict__ acnt,
                                                     int wait_limit, int sleep_after)
{
    using C = AnnealMwG<MS, TT, PD>;
    constexpr int NW = C::NW, NB = C::NB, DW = C::DW, PER = C::PER, P = C::P, SLOTS = C::SLOTS;
    constexpr int MP = 64 * MS;
    constexpr int ROWB = MP * (int)sizeof(TT);                 // bytes per tile row
    constexpr int EB = 8 * (int)sizeof(TT);                    // bits per element
    __shared__ __align__(16) uint8_t own[NW][C::NOFF > 0 ? C::NOFF : 1][C::NOFF > 0 ? C::OBLK : 16];
    __shared__ uint32_t lists[MS][SLOTS];
    __shared__ int64_t esum[NW];
    __shared__ int32_t asum[NW];
    __shared__ int32_t bad;
    const int q = jobs[slot];
    const int base = off[q], m = off[q + 1] - base;
    const uint8_t *gt8 = reinterpret_cast<const uint8_t *>(tiles + tile_off[q]);
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int s0 = w * NB;
    const int r = 0;                                           // one replica per workgroup
    uint8_t *ow = &own[w][0][0];

    // this wave's columns of row x: dword 16 lane + 4 w of the row
    constexpr int LB = C::LB;
    const uint8_t *colp = gt8 + MS * (int)sizeof(TT) * lane + LB * w;
    auto elem_of = [&](uint32_t x, int t) -> int32_t {
        return sizeof(TT) == 1 ? (int32_t)(int8_t)(x >> (8 * t)) : (int32_t)(int16_t)(x >> (16 * t));
    };

    // own rows: diagonal blocks into VGPRs, the upper off-diagonal blocks of
    // the own square into LDS (the lower ones are their transposes)
    // one array per block, so that each is promoted to VGPRs on its own
    uint32_t dc0[DW], dc1[DW], dc2[DW], dc3[DW];
    auto dcol = [&](int j) -> uint32_t (&)[DW] { return j == 0 ? dc0 : j == 1 ? dc1 : j == 2 ? dc2 : dc3; };
    static_assert(NB <= 4, "at most four blocks per wave");
#pragma unroll
    for (int a = 0; a < NB; ++a) {
#pragma unroll 2
        for (int i = 0; i < DW; ++i) {
            uint32_t wv = 0;
#pragma unroll
            for (int p = 0; p < PER; ++p) {
                const int rr = i * PER + p;
                const uint32_t x = load_lb<LB>(colp + (size_t)(64 * (s0 + a) + rr) * ROWB);
                wv |= ((uint32_t)elem_of(x, a) & (0xFFFFFFFFu >> (32 - EB))) << (p * EB);
#pragma unroll
                for (int t = a + 1; t < NB; ++t) {
                    const TT v = (TT)elem_of(x, t);
                    *reinterpret_cast<TT *>(ow + own_pair(a, t, NB) * C::OBLK + rr * C::OSTR + lane * (int)sizeof(TT)) = v;
                }
            }
            dcol(a)[i] = wv;
        }
    }
    for (int t = tid; t < MS * SLOTS; t += blockDim.x) (&lists[0][0])[t] = 0u;
    if (tid == 0) bad = 0;
    __syncthreads();

    int32_t F[NB], M[NB];
    uint64_t active[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int pos = 64 * (s0 + j) + lane;
        F[j] = pos < m ? F0[base + pos] : 0;
        M[j] = (pos < m && y0[base + pos]) ? -1 : 0;
        const int na = min(max(m - 64 * (s0 + j), 0), 64);
        active[j] = na == 64 ? ~0ull : ((1ull << na) - 1ull);
    }
    const uint32_t tag = (1u << 28) | (inst_base + (it ? it->inst : 0u) + (uint32_t)q);
    const int sh = 32 - B;
    auto thresholds = [&](int sw, int32_t (&tv)[NB]) {
        const uint4 o = qb_philox(make_uint4(((uint32_t)(s0 >> 2) << 6) | (uint32_t)lane, (uint32_t)sw, (uint32_t)r, tag),
                                  k0, k1);
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int sq = (s0 + j) & 3;
            const uint32_t uw = sq == 0 ? o.x : sq == 1 ? o.y : sq == 2 ? o.z : o.w;
            tv[j] = thr[((size_t)sw << B) + (uw >> sh)];
        }
    };
    int32_t tvn[NB];
    thresholds(0, tvn);
    int64_t e = 0;
    int32_t nacc = 0;
    int Gc = 0;
    bool ok = true;

    for (int sw = 0; sw < nsw && ok; ++sw) {
        const int G0 = sw * MS + s0;
        for (; Gc < G0; ++Gc) {
            const int sc = Gc & (MS - 1);
            if (sc >= s0 && sc < s0 + NB) continue;       // own list: applied while produced
            const uint32_t want = (uint32_t)(Gc + 1);
            const uint32_t *lst = lists[sc];
            const uint8_t *rowp = colp + (size_t)(64 * sc) * ROWB;
            int idx = 0, spins = 0;
            while (true) {
                uint32_t vv[P];
#pragma unroll
                for (int i = 0; i < P; ++i)
                    vv[i] = (uint32_t)__builtin_amdgcn_readfirstlane(
                        (int)__hip_atomic_load(&lst[idx + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
                int n = 0;
                bool stop = false, end = false;
#pragma unroll
                for (int i = 0; i < P; ++i) {
                    if (!stop) {
                        if ((vv[i] >> 8) != want)
                            stop = true;
                        else if (((vv[i] >> 1) & 127u) == 64u)
                            stop = end = true;
                        else
                            ++n;
                    }
                }
                if (n == 0 && !end) {
                    if (++spins > (LIM ? wait_limit : MW_WAIT_DEFAULT)) {
                        ok = false;
                        break;
                    }
                    if (spins > sleep_after) __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                spins = 0;
                uint32_t x[P];
#pragma unroll
                for (int i = 0; i < P; ++i)
                    if (i < n) x[i] = load_lb<LB>(rowp + (size_t)((vv[i] >> 1) & 63u) * ROWB);
#pragma unroll
                for (int i = 0; i < P; ++i) {
                    if (i < n) {
                        const int32_t d2 = (vv[i] & 1u) ? -2 : 2;
#pragma unroll
                        for (int t = 0; t < NB; ++t) F[t] += d2 * elem_of(x[i], t);
                    }
                }
                idx += n;
                if (end) break;
            }
            if (!ok) break;
        }
        if (!ok) break;

        int32_t tv[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) tv[j] = tvn[j];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int s = s0 + j;
            const int G = G0 + j;
            uint32_t *out = lists[s];
            const uint32_t gtag = (uint32_t)(G + 1) << 8;
            block_esum<TT> ej = 0;
            int c = 0;
            // dE = sigma F itself, the flips applied at the end of the turn, as
            // in the in-LDS kernel
            const int32_t M0 = M[j];
            const int32_t s2 = M0 ? -2 : 2, ns2 = -s2;    // 2 sigma
            int32_t dE = (F[j] ^ M0) - M0;
            // a lane past the block, or at or below the last accept, compares
            // against INT32_MIN, which no dE reaches (|dE| <= |F| <= (2n + 1)
            // max|Q| < 2^31, checked when the problem is created): no mask of
            // pending lanes on the accept chain
            int32_t tk = (active[j] >> lane) & 1ull ? tv[j] : INT32_MIN;
            uint64_t acc = __ballot(dE <= tk);
            const uint64_t ym0 = __ballot(M0 != 0);      // y at the turn's start, as in the in-LDS kernel
            uint64_t amask = 0;
            // the other own blocks' elements of the accepted row: read after
            // the decision, added one accept later (off the accept chain)
            int32_t pt[NB];
            int32_t pd2 = 0;
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) pt[jj] = 0;
            while (acc) {
                const int k = __builtin_ctzll(acc);
                const uint64_t bk = 1ull << k;
                ej += __builtin_amdgcn_readlane(dE, k);
                amask |= bk;
                int32_t f, d2, yk;
                qb_accept_sign<true>(ym0, k, s2, ns2, f, d2, yk);
                dE += __mul24(f, diag_at<TT, DW>(dcol(j), k));
                __hip_atomic_store(&out[c], gtag | ((uint32_t)k << 1) | (uint32_t)yk, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                ++c;
                tk = lane <= k ? INT32_MIN : tk;
                acc = __ballot(dE <= tk);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int jj = 0; jj < NB; ++jj) {
                    if (jj == j) continue;
                    F[jj] += __mul24(pd2, pt[jj]);
                    const int o = jj > j ? own_pair(j, jj, NB) * C::OBLK + k * C::OSTR + lane * (int)sizeof(TT)
                                         : own_pair(jj, j, NB) * C::OBLK + lane * C::OSTR + k * (int)sizeof(TT);
                    pt[jj] = (int32_t)*reinterpret_cast<const TT *>(ow + o);
                }
                pd2 = d2;
            }
#pragma unroll
            for (int jj = 0; jj < NB; ++jj)
                if (jj != j) F[jj] += __mul24(pd2, pt[jj]);
            F[j] = (dE ^ M0) - M0;
            M[j] = (((ym0 ^ amask) >> lane) & 1ull) ? -1 : 0;
            __hip_atomic_store(&out[c], gtag | (64u << 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            e += ej;
            nacc += c;
        }
        Gc = G0 + NB;
        if (sw + 1 < nsw) thresholds(sw + 1, tvn);
    }

    if (!ok && lane == 0) __hip_atomic_store(&bad, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (lane == 0) esum[w] = e;
    if (lane == 0) asum[w] = nacc;
    uint8_t *Yr = Y + (size_t)base * R;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int pos = 64 * (s0 + j) + lane;
        if (pos < m) Yr[pos] = (uint8_t)(M[j] & 1);
    }
    __syncthreads();
    if (tid == 0) {
        int64_t t = 0;
        int32_t na = 0;
        for (int v = 0; v < NW; ++v) {
            t += esum[v];
            na += asum[v];
        }
        eout[(size_t)q * R] = bad ? INT64_MIN : t;
        if (acnt) acnt[(size_t)q * R] = na;
    }
}
template <int MS, typename TT, bool LIM, int PD>
__global__ void __launch_bounds__(256) k_anneal_mw_g(const int32_t *__restrict__ jobs,
                                                     const int32_t *__restrict__ off,
                                                     const int64_t *__restrict__ tile_off,
                                                     const TT *__restrict__ tiles, const int32_t *__restrict__ F0,
                                                     const uint8_t *__restrict__ y0, int nsw, int B,
                                                     const int32_t *__restrict__ thr, int R, uint32_t k0,
                                                     uint32_t k1, uint32_t inst_base, const qb_iter *__restrict__ it, uint8_t *__restrict__ Y,
                                                     int64_t *__restrict__ eout, int32_t *__restrict__ acnt,
                                                     int wait_limit, int sleep_after,
        int *__restrict__ queue, int njobs)
{
    __shared__ int slot_s;
    for (int pass = 0;; ++pass) {
        const int slot = qb_next_slot(queue, njobs, pass, &slot_s);
        if (slot < 0) break;
        anneal_mw_g_job<MS, TT, LIM, PD>(slot, jobs, off, tile_off, tiles, F0, y0, nsw, B, thr, R, k0, k1, inst_base, it, Y, eout, acnt, wait_limit, sleep_after);
        __syncthreads();   // the next job reuses the workgroup's LDS
    }
}


template <int MS, typename TT, int PD>
void launch_mw_g_depth(int nblocks, int lim, hipStream_t s, const int32_t *jobs, qb_batch b, const void *tiles,
                       const int32_t *F0, const uint8_t *y0, int nsw, int B, const int32_t *thr, int R, uint64_t seed,
                       uint32_t inst_base, const qb_iter *it, uint8_t *Y, int64_t *e)
{
    constexpr int NT = 64 * AnnealMwG<MS, TT, PD>::NW;
    if (lim == MW_WAIT_DEFAULT)
        k_anneal_mw_g<MS, TT, false, PD><<<qb_grid(b, nblocks), NT, 0, s>>>(
            jobs, b->off_d, b->tile_off_d, (const TT *)tiles, F0, y0, nsw, B, thr, R, (uint32_t)seed,
            (uint32_t)(seed >> 32), inst_base, it, Y, e, b->acnt_d, lim, b->plan.sleep_after, b->lq, nblocks);
    else
        k_anneal_mw_g<MS, TT, true, PD><<<qb_grid(b, nblocks), NT, 0, s>>>(
            jobs, b->off_d, b->tile_off_d, (const TT *)tiles, F0, y0, nsw, B, thr, R, (uint32_t)seed,
            (uint32_t)(seed >> 32), inst_base, it, Y, e, b->acnt_d, lim, b->plan.sleep_after, b->lq, nblocks);
}

template <int MS, typename TT>
bool launch_anneal_mw_g(int nblocks, int R, hipStream_t s, const int32_t *jobs, qb_batch b, const void *tiles,
                        const int32_t *F0, const uint8_t *y0, int nsw, int B, const int32_t *thr, uint64_t seed,
                        uint32_t inst_base, const qb_iter *it, uint8_t *Y, int64_t *e)
{
    if (R != 1 || (int64_t)nsw * MS + 1 >= (int64_t(1) << 24)) return false;
    const int32_t lim = g_wait_limit.load(std::memory_order_relaxed);
    switch (b->plan.depth) {
    case 16: launch_mw_g_depth<MS, TT, 16>(nblocks, lim, s, jobs, b, tiles, F0, y0, nsw, B, thr, R, seed, inst_base,
                                           it, Y, e); break;
    case 32: launch_mw_g_depth<MS, TT, 32>(nblocks, lim, s, jobs, b, tiles, F0, y0, nsw, B, thr, R, seed, inst_base,
                                           it, Y, e); break;
    default: launch_mw_g_depth<MS, TT, 8>(nblocks, lim, s, jobs, b, tiles, F0, y0, nsw, B, thr, R, seed, inst_base,
                                          it, Y, e); break;
    }
    return true;
}

// ------------------------------------------------- anneal, one wave, couplings in registers
// One replica per wave again (the R replicas of a job share a workgroup and
// its tile in LDS), with the multi-wave owner's accept chain: lane L holds
// column L of the current diagonal 64 x 64 block, T[64 s + k][64 s + L] for
// k < 64, in VGPRs, and the block's move values dE = sigma F are updated
// from there, so no memory access is on the chain.  The accepted row's
// elements in the other blocks (one LDS read of the lane's slice) are added
// to their F one accept late, after the next accept's chain, and the last
// one at the end of the block.  No wave waits on another: a sweep has no
// hand-off between waves.  By symmetry column L of a diagonal block is its
// row L; with the symmetric-block placement (mp = 512, int8) that row is
// read straight from the stored diagonal block, otherwise (whole tile in
// LDS) the kernel first copies the diagonal blocks as [block][L][k] rows.
template <int MS, typename TT, int MODE>
struct AnnealDc {
    static constexpr int MP = 64 * MS;
    static constexpr size_t tile = MODE == 0 ? (size_t)MP * MP * sizeof(TT) : SYM_BYTES;
    static constexpr size_t dcol = MODE == 0 ? (size_t)MS * 64 * 64 * sizeof(TT) : 0;
    static constexpr int DW = 64 * (int)sizeof(TT) / 4;
    static constexpr bool fits = tile + dcol + 256 <= (size_t)MW_LDS_LIMIT;
};

template <int MS, typename TT, int MODE>
__device__ __forceinline__ void anneal_dc_job(int slot, const int32_t *__restrict__ jobs, const int32_t *__restrict__ off,
                                                    const int64_t *__restrict__ tile_off,
                                                    const TT *__restrict__ tiles, const int32_t *__restrict__ F0,
                                                    const uint8_t *__restrict__ y0, int nsw, int B,
                                                    const int32_t *__restrict__ thr, int R, uint32_t k0,
                                                    uint32_t k1, uint32_t inst_base, const qb_iter *__restrict__ it,
                                                    uint8_t *__restrict__ Y, int64_t *__restrict__ eout,
                                                    int32_t *__restrict__ acnt)
{
    using C = AnnealDc<MS, TT, MODE>;
    constexpr int MP = C::MP, DW = C::DW;
    static_assert(C::fits, "tile and columns must fit LDS");
    __shared__ __align__(16) uint8_t lds[C::tile + (C::dcol ? C::dcol : 16)];
    const int q = jobs[slot];
    const int base = off[q], m = off[q + 1] - base;
    const TT *gtile = tiles + tile_off[q];
    const int tid = threadIdx.x, lane = tid & 63, r = tid >> 6;

    if constexpr (MODE == 0) {
        constexpr int n16 = (int)(C::tile / 16);
        const uint4 *src = reinterpret_cast<const uint4 *>(gtile);
        uint4 *dst = reinterpret_cast<uint4 *>(lds);
        for (int t = tid; t < n16; t += blockDim.x) dst[t] = src[t];
        // diagonal blocks as rows: [b][L][k] = T[64 b + L][64 b + k]
        TT *dc = reinterpret_cast<TT *>(lds + C::tile);
        for (int t = tid; t < MS * 4096; t += blockDim.x) {
            const int bk = t >> 12, L = (t >> 6) & 63, k = t & 63;
            dc[t] = gtile[(size_t)(64 * bk + L) * MP + k * MS + bk];
        }
        __syncthreads();
    } else {
        const uint64_t *src = reinterpret_cast<const uint64_t *>(gtile);
        for (int t = tid; t < MP * 64; t += blockDim.x) {
            const int x = t >> 6, cc = t & 63;
            const uint64_t w = src[t];
            const int a = x >> 6, rr = x & 63;
#pragma unroll
            for (int b = 0; b < 8; ++b)
                if (b >= a) lds[sym_block_index(a, b) * SYM_BLOCK + rr * SYM_STRIDE + cc] = (uint8_t)(w >> (8 * b));
        }
        __syncthreads();
    }
    if (r >= R) return;   // no barrier follows

    int32_t F[MS];
    uint32_t ybits = 0;
#pragma unroll
    for (int s = 0; s < MS; ++s) {
        const int pos = 64 * s + lane;
        F[s] = pos < m ? F0[base + pos] : 0;
        if (pos < m && y0[base + pos]) ybits |= 1u << s;
    }
    // row L of diagonal block s (its column L by symmetry)
    auto column = [&](int s, uint32_t (&d)[DW]) {
        const uint32_t *src;
        if constexpr (MODE == 0)
            src = reinterpret_cast<const uint32_t *>(lds + C::tile + ((size_t)s * 64 + lane) * 64 * sizeof(TT));
        else
            src = reinterpret_cast<const uint32_t *>(lds + sym_block_index(s, s) * SYM_BLOCK + lane * SYM_STRIDE);
#pragma unroll
        for (int i = 0; i < DW; ++i) d[i] = src[i];
    };
    int64_t e = 0;
    int32_t nacc = 0;
    const uint32_t tag = (1u << 28) | (inst_base + (it ? it->inst : 0u) + (uint32_t)q);
    constexpr int G = (MS + 3) / 4;
    const int sh = 32 - B;
    auto thresholds = [&](int sw, int32_t (&tv)[MS]) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint4 o = qb_philox(make_uint4(((uint32_t)g << 6) | (uint32_t)lane, (uint32_t)sw, (uint32_t)r, tag),
                                      k0, k1);
            const int32_t *ts = thr + ((size_t)sw << B);
#pragma unroll
            for (int w = 0; w < 4; ++w)
                if (4 * g + w < MS) tv[4 * g + w] = ts[qb_word(o, w) >> sh];
        }
    };
    int32_t tvn[MS];
    thresholds(0, tvn);

    for (int sw = 0; sw < nsw; ++sw) {
        int32_t tv[MS];
#pragma unroll
        for (int s = 0; s < MS; ++s) tv[s] = tvn[s];
        if (sw + 1 < nsw) thresholds(sw + 1, tvn);
#pragma unroll
        for (int s = 0; s < MS; ++s) {
            const int na = min(max(m - 64 * s, 0), 64);
            if (na == 0) continue;
            uint64_t pend = na == 64 ? ~0ull : ((1ull << na) - 1ull);
            uint32_t dcl[DW];
            column(s, dcl);
            const int32_t M0 = ((ybits >> s) & 1u) ? -1 : 0;
            const int32_t s2 = M0 ? -2 : 2, ns2 = -s2;   // 2 sigma
            int32_t dE = (F[s] ^ M0) - M0;
            const uint64_t ym0 = __ballot(M0 != 0);      // y at the block's start (a lane accepts once)
            uint64_t amask = 0;                          // lanes accepted in the block
            block_esum<TT> eb = 0;
            uint64_t acc = __ballot(dE <= tv[s]) & pend;
            int32_t pr[MS];
            int32_t pd2 = 0;                             // 0: nothing pending
            while (acc) {
                const int k = __builtin_ctzll(acc);
                const uint64_t bk = 1ull << k;
                eb += __builtin_amdgcn_readlane(dE, k);
                amask |= bk;
                int32_t f, d2, yk;
                qb_accept_sign<false>(ym0, k, s2, ns2, f, d2, yk);
                dE += __mul24(f, diag_at<TT, DW>(dcl, k));
                pend &= (~0ull << k) << 1;
                const uint64_t accn = __ballot(dE <= tv[s]) & pend;
                // the chain is done: add the previous accepted row to the
                // other blocks, then read this one
                __builtin_amdgcn_sched_barrier(0);
                if (pd2) {
#pragma unroll
                    for (int s3 = 0; s3 < MS; ++s3)
                        if (s3 != s) F[s3] += __mul24(pd2, pr[s3]);
                }
                fetch_row<MS, TT, MODE>(lds, gtile, 64 * s + k, lane, pr);
                pd2 = d2;
                acc = accn;
            }
            if (pd2) {
#pragma unroll
                for (int s3 = 0; s3 < MS; ++s3)
                    if (s3 != s) F[s3] += __mul24(pd2, pr[s3]);
            }
            F[s] = (dE ^ M0) - M0;
            e += eb;
            nacc += __builtin_popcountll(amask);
            if (((ym0 ^ amask) >> lane) & 1ull)
                ybits |= 1u << s;
            else
                ybits &= ~(1u << s);
        }
    }

    uint8_t *Yr = Y + (size_t)base * R + (size_t)r * m;
#pragma unroll
    for (int s = 0; s < MS; ++s) {
        const int pos = 64 * s + lane;
        if (pos < m) Yr[pos] = (uint8_t)((ybits >> s) & 1u);
    }
    if (lane == 0) eout[(size_t)q * R + r] = e;
    if (acnt && lane == 0) acnt[(size_t)q * R + r] = nacc;
}
template <int MS, typename TT, int MODE>
__global__ void __launch_bounds__(1024) k_anneal_dc(const int32_t *__restrict__ jobs, const int32_t *__restrict__ off,
                                                    const int64_t *__restrict__ tile_off,
                                                    const TT *__restrict__ tiles, const int32_t *__restrict__ F0,
                                                    const uint8_t *__restrict__ y0, int nsw, int B,
                                                    const int32_t *__restrict__ thr, int R, uint32_t k0,
                                                    uint32_t k1, uint32_t inst_base, const qb_iter *__restrict__ it,
                                                    uint8_t *__restrict__ Y, int64_t *__restrict__ eout,
                                                    int32_t *__restrict__ acnt,
        int *__restrict__ queue, int njobs)
{
    __shared__ int slot_s;
    for (int pass = 0;; ++pass) {
        const int slot = qb_next_slot(queue, njobs, pass, &slot_s);
        if (slot < 0) break;
        anneal_dc_job<MS, TT, MODE>(slot, jobs, off, tile_off, tiles, F0, y0, nsw, B, thr, R, k0, k1, inst_base, it, Y, eout, acnt);
        __syncthreads();   // the next job reuses the workgroup's LDS
    }
}


template <int MS, typename TT, int MODE>
bool launch_anneal_dc(int nblocks, int R, hipStream_t s, const int32_t *jobs, qb_batch b, const void *tiles,
                      const int32_t *F0, const uint8_t *y0, int nsw, int B, const int32_t *thr, uint64_t seed,
                      uint32_t inst_base, const qb_iter *it, uint8_t *Y, int64_t *e)
{
    if constexpr (!AnnealDc<MS, TT, MODE>::fits) {
        return false;
    } else {
        k_anneal_dc<MS, TT, MODE><<<qb_grid(b, nblocks), 64 * R, 0, s>>>(jobs, b->off_d, b->tile_off_d,
                                                                          (const TT *)tiles, F0, y0, nsw, B, thr, R,
                                                                          (uint32_t)seed, (uint32_t)(seed >> 32),
                                                                          inst_base, it, Y, e, b->acnt_d, b->lq,
                                                                          nblocks);
        return true;
    }
}

__global__ void k_reset_queues(int *__restrict__ q, int n)
{
    if ((int)threadIdx.x < n) q[threadIdx.x] = 0;
}

bool dispatch_anneal(int cls, bool int8_tile, int nblocks, int R, hipStream_t s, const int32_t *jobs, qb_batch b,
                     const void *tiles, const int32_t *F0, const uint8_t *y0, int nsw, int B, const int32_t *thr,
                     uint64_t seed, uint32_t inst_base, const qb_iter *it, uint8_t *Y, int64_t *e)
{
#define QB_ARGS nblocks, R, s, jobs, b, tiles, F0, y0, nsw, B, thr, seed, inst_base, it, Y, e
    // the multi-wave kernel with rows in global memory, where the plan asks for it
    if (b->plan.kernel[cls] == QB_ANNEAL_MULTI_WAVE_GLOBAL) {
        if (int8_tile) {
            switch (cls) {
            case 1: if (launch_anneal_mw_g<8, int8_t>(QB_ARGS)) return true; break;
            case 2: if (launch_anneal_mw_g<4, int8_t>(QB_ARGS)) return true; break;
            case 3: if (launch_anneal_mw_g<2, int8_t>(QB_ARGS)) return true; break;
            }
        } else {
            switch (cls) {
            case 2: if (launch_anneal_mw_g<4, int16_t>(QB_ARGS)) return true; break;
            case 3: if (launch_anneal_mw_g<2, int16_t>(QB_ARGS)) return true; break;
            }
        }
    }
    // the one-wave kernel with the couplings in registers, where the plan asks for it
    if (b->plan.kernel[cls] == QB_ANNEAL_ONE_WAVE_REG) {
        if (int8_tile) {
            switch (cls) {
            case 1: if (launch_anneal_dc<8, int8_t, 1>(QB_ARGS)) return true; break;
            case 2: if (launch_anneal_dc<4, int8_t, 0>(QB_ARGS)) return true; break;
            case 3: if (launch_anneal_dc<2, int8_t, 0>(QB_ARGS)) return true; break;
            case 4: if (launch_anneal_dc<1, int8_t, 0>(QB_ARGS)) return true; break;
            }
        } else {
            switch (cls) {
            case 3: if (launch_anneal_dc<2, int16_t, 0>(QB_ARGS)) return true; break;
            case 4: if (launch_anneal_dc<1, int16_t, 0>(QB_ARGS)) return true; break;
            }
        }
    }
    // the multi-wave kernel where its replicas fit one workgroup
    if (b->plan.kernel[cls] != QB_ANNEAL_ONE_WAVE && int8_tile) {
        switch (cls) {
        case 0: if (launch_anneal_mw_g<16, int8_t>(QB_ARGS)) return true; break;
        case 1: if (launch_anneal_mw<8, int8_t, 1>(QB_ARGS)) return true; break;
        case 2: if (launch_anneal_mw<4, int8_t, 0>(QB_ARGS)) return true; break;
        case 3: if (launch_anneal_mw<2, int8_t, 0>(QB_ARGS)) return true; break;
        }
    } else if (b->plan.kernel[cls] != QB_ANNEAL_ONE_WAVE) {
        switch (cls) {
        case 1: if (launch_anneal_mw_g<8, int16_t>(QB_ARGS)) return true; break;
        case 2: if (launch_anneal_mw<4, int16_t, 0>(QB_ARGS)) return true; break;
        case 3: if (launch_anneal_mw<2, int16_t, 0>(QB_ARGS)) return true; break;
        }
    }
    if (int8_tile) {
        switch (cls) {
        case 0: launch_anneal<16, int8_t, 2>(QB_ARGS); return true;
        case 1: launch_anneal<8, int8_t, 1>(QB_ARGS); return true;
        case 2: launch_anneal<4, int8_t, 0>(QB_ARGS); return true;
        case 3: launch_anneal<2, int8_t, 0>(QB_ARGS); return true;
        case 4: launch_anneal<1, int8_t, 0>(QB_ARGS); return true;
        }
    } else {
        switch (cls) {
        case 0: launch_anneal<16, int16_t, 2>(QB_ARGS); return true;
        case 1: launch_anneal<8, int16_t, 2>(QB_ARGS); return true;
        case 2: launch_anneal<4, int16_t, 0>(QB_ARGS); return true;
        case 3: launch_anneal<2, int16_t, 0>(QB_ARGS); return true;
        case 4: launch_anneal<1, int16_t, 0>(QB_ARGS); return true;
        }
    }
#undef QB_ARGS
    return false;
}

// ------------------------------------------------------------------ write-back
__global__ void __launch_bounds__(256) k_writeback(int n, int R, const int32_t *__restrict__ sol,
                                                   const int32_t *__restrict__ off, const int32_t *__restrict__ idx,
                                                   const uint8_t *__restrict__ Y, const int64_t *__restrict__ e,
                                                   const uint8_t *__restrict__ y0, uint8_t *__restrict__ X,
                                                   int8_t *__restrict__ dX, int64_t *__restrict__ ebest,
                                                   int not_worse, int32_t *__restrict__ status)
{
    const int q = blockIdx.x;
    const int base = off[q], m = off[q + 1] - base, p = sol[q];
    bool failed;
    const int rb = qb_best_replica(e + (size_t)q * R, R, &failed);
    if (failed && threadIdx.x == 0) atomicOr(status, QB_FLAG_STATE);
    if (ebest && threadIdx.x == 0) ebest[q] = rb < 0 ? INT64_MIN : e[(size_t)q * R + rb];
    if (rb < 0) return;                                    // no replica finished: x_S and dX stay
    if (not_worse && e[(size_t)q * R + rb] > 0) return;   // x_S and dX stay as they are
    const uint8_t *Yr = Y + (size_t)base * R + (size_t)rb * m;
    for (int a = threadIdx.x; a < m; a += 256) {
        const int j = idx[base + a];
        const uint8_t y = Yr[a];
        X[(int64_t)p * n + j] = y;
        dX[(int64_t)p * n + j] = (int8_t)((int)y - (int)y0[base + a]);
    }
}

}  // namespace

extern "C" qb_status qb_extract(qb_problem P, qb_batch b, const uint8_t *X_d, const int32_t *H_d, void *tile_d,
                               int32_t *c_d, int32_t *F0_d, uint8_t *y0_d, void *stream)
{
    if (!P || !b || !X_d || !H_d || !tile_d || !F0_d || !y0_d) return QB_E_ARG;
    if (b->n != P->n) return QB_E_ARG;
    if (P->sparse) return QB_E_UNSUPPORTED;
    if ((uintptr_t)tile_d & 15) return QB_E_ARG;
    if (b->J == 0) return QB_OK;
    hipStream_t s = qb_stream(stream);
    if (P->int8_ok)
        k_extract<int8_t><<<b->J, EXTRACT_THREADS, 0, s>>>(P->Q, P->Q8, P->n, b->sol_d, b->off_d, b->tile_off_d, b->idx_d,
                                               X_d, H_d, (int8_t *)tile_d, c_d, F0_d, y0_d);
    else
        k_extract<int16_t><<<b->J, EXTRACT_THREADS, 0, s>>>(P->Q, P->Q, P->n, b->sol_d, b->off_d, b->tile_off_d, b->idx_d,
                                                X_d, H_d, (int16_t *)tile_d, c_d, F0_d, y0_d);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

qb_status qb_anneal_x(qb_batch b, const void *tile_d, int32_t int8_tile, const int32_t *F0_d, const uint8_t *y0_d,
                      int32_t nsw, int32_t B, const int32_t *thr_d, int32_t R, uint64_t seed, uint32_t inst_base,
                      const qb_iter *it, uint8_t *Y_d, int64_t *e_d, void *stream)
{
    if (!b || !tile_d || !F0_d || !y0_d || !thr_d || !Y_d || !e_d) return QB_E_ARG;
    if (nsw < 1 || B < 1 || B > 16 || R < 1 || R > 16) return QB_E_ARG;
    if ((uintptr_t)tile_d & 15) return QB_E_ARG;
    if ((uint64_t)inst_base + (uint64_t)b->J > (1ull << 28)) return QB_E_RANGE;
    hipStream_t s = qb_stream(stream);
    // every size class starts at once: the fork precedes the first launch
    int ncls = 0;
    for (int c = 0; c < QB_NCLASS; ++c) ncls += b->cls_end[c] > b->cls_begin[c];
    if (ncls == 0) return QB_OK;
    const bool persist = b->plan.persistent != 0;
    if (persist) {
        k_reset_queues<<<1, 64, 0, s>>>(b->queue_d, QB_NCLASS);
        QB_LAUNCH_CHECK();
    }
    if (ncls > 1) QB_TRY_HIP(hipEventRecord(b->ev_fork, s));
    int ncu = 0;
    if (persist) QB_TRY_HIP(qb_cu_count(&ncu));
    bool first = true;
    for (int c = 0; c < QB_NCLASS; ++c) {
        const int nblk = b->cls_end[c] - b->cls_begin[c];
        if (nblk <= 0) continue;
        hipStream_t ls = s;
        if (!first) {
            ls = b->side[c];
            QB_TRY_HIP(hipStreamWaitEvent(ls, b->ev_fork, 0));
        }
        // persistent: a grid of workgroups pulls the class's jobs from its queue
        b->lq = persist ? b->queue_d + c : nullptr;
        b->lgrid = persist ? std::min(nblk, std::max(1, ncu * b->plan.wgs_per_cu)) : 0;
        const int32_t *order = (b->plan.lpt ? b->lpt_d : b->iord_d) + b->cls_begin[c];
        const bool ok = dispatch_anneal(c, int8_tile != 0, nblk, R, ls, order, b, tile_d, F0_d, y0_d, nsw, B, thr_d,
                                        seed, inst_base, it, Y_d, e_d);
        b->lq = nullptr;
        b->lgrid = 0;
        if (!ok) return QB_E_UNSUPPORTED;
        QB_LAUNCH_CHECK();
        if (!first) {
            QB_TRY_HIP(hipEventRecord(b->ev_join[c], ls));
            QB_TRY_HIP(hipStreamWaitEvent(s, b->ev_join[c], 0));
        }
        first = false;
    }
    return QB_OK;
}

extern "C" qb_status qb_anneal(qb_batch b, const void *tile_d, int32_t int8_tile, const int32_t *F0_d,
                              const uint8_t *y0_d, int32_t nsw, int32_t B, const int32_t *thr_d, int32_t R,
                              uint64_t seed, uint32_t inst_base, uint8_t *Y_d, int64_t *e_d, void *stream)
{
    return qb_anneal_x(b, tile_d, int8_tile, F0_d, y0_d, nsw, B, thr_d, R, seed, inst_base, nullptr, Y_d, e_d, stream);
}

extern "C" qb_status qb_writeback(qb_batch b, int32_t R, const uint8_t *Y_d, const int64_t *e_d,
                                 const uint8_t *y0_d, uint8_t *X_d, int8_t *dX_d, int64_t *ebest_job_d,
                                 int32_t flags, void *stream)
{
    if (!b || R < 1 || R > 16 || !Y_d || !e_d || !y0_d || !X_d || !dX_d || (flags & ~1)) return QB_E_ARG;
    if (b->J == 0) return QB_OK;
    k_writeback<<<b->J, 256, 0, qb_stream(stream)>>>(b->n, R, b->sol_d, b->off_d, b->idx_d, Y_d, e_d, y0_d, X_d,
                                                     dX_d, ebest_job_d, flags & 1, b->status_d);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

extern "C" qb_status qb_set_anneal_wait_limit(int32_t polls)
{
    if (polls < 0) return QB_E_ARG;
    g_wait_limit.store(polls, std::memory_order_relaxed);
    return QB_OK;
}
