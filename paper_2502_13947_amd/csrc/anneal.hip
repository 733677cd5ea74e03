// Sub-QUBO extraction (eq. 4, Alg. 3 lines 3-5), the batched Ising-machine
// stage (Alg. 3 line 6) and the write-back (Alg. 3 line 7) on gfx950.
//
// Annealer layout: one replica per wave64, the R replicas of a job share a
// workgroup and its tile.  Lane L owns positions 64*s + L (s < MS = mp/64):
// their flip bases F live in VGPRs and their spins in a per-lane bit mask.
// A sweep visits blocks of 64 positions; all 64 uniforms and thresholds of a
// block are ready before the block starts, the accept predicate is evaluated
// by every pending lane at once, and the lowest accepting lane k is taken
// (ballot + find-first-set).  After flipping k every lane adds 2 d T[k][own]
// to its F (one row read per accept) and only lanes after k re-evaluate:
// lanes before k were rejected with exactly the fields the sequential sweep
// would have shown them, so the result is the sequential sweep's, bit for
// bit, with #accepts + MS ballot rounds per sweep instead of m steps.
//
// Tile placement by size class: mp <= 256 (int8) or <= 256 (int16): whole
// tile in LDS; mp = 512 int8: the 36 upper 64x64 blocks of the symmetric tile
// in LDS (156,672 bytes, rows padded to 68 bytes so that both row and column
// reads of a block are bank-conflict free); otherwise rows stream from L2/HBM.
#include "qb_internal.h"

namespace {

// ------------------------------------------------------------------ extract
template <typename TT>
__global__ void __launch_bounds__(256) k_extract(const int16_t *__restrict__ Q16, const TT *__restrict__ Qt,
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
    const int q = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int base = off[q], m = off[q + 1] - base, p = sol[q];
    const int MS = qb_tile_ms(m), MP = MS * 64;
    const int64_t xo = (int64_t)p * n;
    for (int a = tid; a < m; a += 256) {
        const int j = idx[base + a];
        S[a] = j;
        ys[a] = X[xo + j];
    }
    __syncthreads();
    for (int a = tid; a < m; a += 256) {
        const int i = S[a];
        const int32_t qii = Q16[(int64_t)i * n + i];
        F0[base + a] = qii + 2 * (H[xo + i] - qii * (int32_t)ys[a]);
        y0[base + a] = ys[a];
    }
    TT *tile = tiles + tile_off[q];
    for (int a = wid; a < MP; a += 4) {
        const bool arow = a < m;
        const TT *qrow = Qt + (arow ? (int64_t)S[a] * n : 0);
        int32_t rowsum = 0;
        for (int s = 0; s < MS; ++s) {
            const int b = 64 * s + lane;
            int32_t v = 0;
            if (arow && b < m && b != a) v = qrow[S[b]];
            tile[(int64_t)a * MP + lane * MS + s] = (TT)v;
            if (b < m) rowsum += v * (int32_t)ys[b];
        }
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

// ------------------------------------------------------------------ anneal
constexpr int SYM_STRIDE = 68;                   // bytes per row of a stored 64x64 block
constexpr int SYM_BLOCK = 64 * SYM_STRIDE;       // 4352
constexpr int SYM_BYTES = 36 * SYM_BLOCK;        // 156,672

__device__ __forceinline__ int sym_block_index(int a, int b)   // a <= b < 8
{
    return a * 8 - (a * (a - 1)) / 2 + (b - a);
}

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
__global__ void __launch_bounds__(1024) k_anneal(const int32_t *__restrict__ jobs, const int32_t *__restrict__ off,
                                                 const int64_t *__restrict__ tile_off,
                                                 const TT *__restrict__ tiles, const int32_t *__restrict__ F0,
                                                 const uint8_t *__restrict__ y0, int nsw, int B,
                                                 const int32_t *__restrict__ thr, int R, uint32_t k0,
                                                 uint32_t k1, uint32_t inst_base, uint8_t *__restrict__ Y,
                                                 int64_t *__restrict__ eout)
{
    constexpr int MP = 64 * MS;
    __shared__ __align__(16) uint8_t lds[AnnealLds<MS, TT, MODE>::bytes];
    const int q = jobs[blockIdx.x];
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
    const uint32_t tag = (1u << 28) | (inst_base + (uint32_t)q);
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
            while (true) {
                const uint32_t yb = (ybits >> s) & 1u;
                const int32_t dE = yb ? -F[s] : F[s];
                const uint64_t acc = __ballot(dE <= tv[s]) & pend;
                if (acc == 0) break;
                const int k = __builtin_ctzll(acc);
                const int32_t dEk = __builtin_amdgcn_readlane(dE, k);
                const int32_t ykb = __builtin_amdgcn_readlane((int32_t)yb, k);
                e += dEk;
                const int32_t d2 = ykb ? -2 : 2;
                if (lane == k) ybits ^= 1u << s;
                int32_t rv[MS];
                fetch_row<MS, TT, MODE>(lds, gtile, 64 * s + k, lane, rv);
#pragma unroll
                for (int s2 = 0; s2 < MS; ++s2) F[s2] += d2 * rv[s2];
                pend &= ~((2ull << k) - 1ull);
            }
        }
    }

    uint8_t *Yr = Y + (size_t)base * R + (size_t)r * m;
#pragma unroll
    for (int s = 0; s < MS; ++s) {
        const int pos = 64 * s + lane;
        if (pos < m) Yr[pos] = (uint8_t)((ybits >> s) & 1u);
    }
    if (lane == 0) eout[(size_t)q * R + r] = e;
}

template <int MS, typename TT, int MODE>
void launch_anneal(int nblocks, int R, hipStream_t s, const int32_t *jobs, qb_batch b, const void *tiles,
                   const int32_t *F0, const uint8_t *y0, int nsw, int B, const int32_t *thr, uint64_t seed,
                   uint32_t inst_base, uint8_t *Y, int64_t *e)
{
    k_anneal<MS, TT, MODE><<<nblocks, 64 * R, 0, s>>>(jobs, b->off_d, b->tile_off_d, (const TT *)tiles, F0, y0,
                                                      nsw, B, thr, R, (uint32_t)seed, (uint32_t)(seed >> 32),
                                                      inst_base, Y, e);
}

bool dispatch_anneal(int cls, bool int8_tile, int nblocks, int R, hipStream_t s, const int32_t *jobs, qb_batch b,
                     const void *tiles, const int32_t *F0, const uint8_t *y0, int nsw, int B, const int32_t *thr,
                     uint64_t seed, uint32_t inst_base, uint8_t *Y, int64_t *e)
{
#define QB_ARGS nblocks, R, s, jobs, b, tiles, F0, y0, nsw, B, thr, seed, inst_base, Y, e
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
                                                   int not_worse)
{
    const int q = blockIdx.x;
    const int base = off[q], m = off[q + 1] - base, p = sol[q];
    int rb = 0;
    for (int r = 1; r < R; ++r)
        if (e[(size_t)q * R + r] < e[(size_t)q * R + rb]) rb = r;
    if (ebest && threadIdx.x == 0) ebest[q] = e[(size_t)q * R + rb];
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
        k_extract<int8_t><<<b->J, 256, 0, s>>>(P->Q, P->Q8, P->n, b->sol_d, b->off_d, b->tile_off_d, b->idx_d,
                                               X_d, H_d, (int8_t *)tile_d, c_d, F0_d, y0_d);
    else
        k_extract<int16_t><<<b->J, 256, 0, s>>>(P->Q, P->Q, P->n, b->sol_d, b->off_d, b->tile_off_d, b->idx_d,
                                                X_d, H_d, (int16_t *)tile_d, c_d, F0_d, y0_d);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

extern "C" qb_status qb_anneal(qb_batch b, const void *tile_d, int32_t int8_tile, const int32_t *F0_d,
                              const uint8_t *y0_d, int32_t nsw, int32_t B, const int32_t *thr_d, int32_t R,
                              uint64_t seed, uint32_t inst_base, uint8_t *Y_d, int64_t *e_d, void *stream)
{
    if (!b || !tile_d || !F0_d || !y0_d || !thr_d || !Y_d || !e_d) return QB_E_ARG;
    if (nsw < 1 || B < 1 || B > 16 || R < 1 || R > 16) return QB_E_ARG;
    if ((uintptr_t)tile_d & 15) return QB_E_ARG;
    if ((uint64_t)inst_base + (uint64_t)b->J > (1ull << 28)) return QB_E_RANGE;
    hipStream_t s = qb_stream(stream);
    bool first = true, forked = false;
    for (int c = 0; c < QB_NCLASS; ++c) {
        const int nblk = b->cls_end[c] - b->cls_begin[c];
        if (nblk <= 0) continue;
        hipStream_t ls = s;
        if (!first) {
            if (!forked) {
                QB_TRY_HIP(hipEventRecord(b->ev_fork, s));
                forked = true;
            }
            ls = b->side[c];
            QB_TRY_HIP(hipStreamWaitEvent(ls, b->ev_fork, 0));
        }
        if (!dispatch_anneal(c, int8_tile != 0, nblk, R, ls, b->lpt_d + b->cls_begin[c], b, tile_d, F0_d, y0_d,
                             nsw, B, thr_d, seed, inst_base, Y_d, e_d))
            return QB_E_UNSUPPORTED;
        QB_LAUNCH_CHECK();
        if (!first) {
            QB_TRY_HIP(hipEventRecord(b->ev_join[c], ls));
            QB_TRY_HIP(hipStreamWaitEvent(s, b->ev_join[c], 0));
        }
        first = false;
    }
    return QB_OK;
}

extern "C" qb_status qb_writeback(qb_batch b, int32_t R, const uint8_t *Y_d, const int64_t *e_d,
                                 const uint8_t *y0_d, uint8_t *X_d, int8_t *dX_d, int64_t *ebest_job_d,
                                 int32_t flags, void *stream)
{
    if (!b || R < 1 || R > 16 || !Y_d || !e_d || !y0_d || !X_d || !dX_d || (flags & ~1)) return QB_E_ARG;
    if (b->J == 0) return QB_OK;
    k_writeback<<<b->J, 256, 0, qb_stream(stream)>>>(b->n, R, b->sol_d, b->off_d, b->idx_d, Y_d, e_d, y0_d, X_d,
                                                     dX_d, ebest_job_d, flags & 1);
    QB_LAUNCH_CHECK();
    return QB_OK;
}
