// Sparse sub-QUBOs: extraction into a per-job ELL (eq. 4, sub-QUBO
// construction in Alg. 3) and the batched Ising-machine stage of Alg. 3 on it,
// on gfx950.
//
// The annealer is the dense kernel's ballot-block sweep with the same
// random numbers and thresholds, so Y and e are bit-identical to it: lane L
// owns positions 64*s + L, a block's 64 candidates are evaluated at once and
// the lowest accepting lane k is taken (ballot + find-first-set), after
// which only lanes past k re-evaluate.  What differs is where the fields
// live and how an accept updates them.  Row k of a sparse tile has a handful
// of entries, so instead of every lane adding its slice of a dense row, the
// flip bases F of each replica live in LDS and lane t adds the t-th entry of
// row k to F[col_t] with one LDS atomic add (the entries of a row have
// distinct columns); the current block's F is read back before the next
// ballot, together with the row of the next lane that accepted in the
// current ballot (most often the next accept).  The job's ELL tile is staged
// in LDS once and shared by the rw replicas (waves) of the workgroup; rw only
// changes the schedule.
#include "qb_internal.h"

namespace {

constexpr int DBLK_BYTES = 64 * 64;   // one diagonal block, int8

// ------------------------------------------------------------------ extract
// One workgroup per job, one thread per row: the entries of Q's row S_a whose
// column is in S (binary search in the ascending index set) become the row's
// ELL words with local column indices; c and F0 as in the dense extraction.
__global__ void __launch_bounds__(256) k_extract_ell(const uint32_t *__restrict__ ell, int W,
                                                     const int32_t *__restrict__ ecnt,
                                                     const int32_t *__restrict__ diag, int n,
                                                     const int32_t *__restrict__ sol,
                                                     const int32_t *__restrict__ off,
                                                     const int32_t *__restrict__ idx,
                                                     const uint8_t *__restrict__ X,
                                                     const int32_t *__restrict__ H, uint32_t *__restrict__ tiles,
                                                     int32_t *__restrict__ c, int32_t *__restrict__ F0,
                                                     uint8_t *__restrict__ y0, uint8_t *__restrict__ dblk,
                                                     const int32_t *__restrict__ dboff)
{
    __shared__ int32_t S[1024];
    __shared__ uint8_t ys[1024];
    const int q = blockIdx.x, tid = threadIdx.x;
    const int base = off[q], m = off[q + 1] - base, p = sol[q];
    const int64_t xo = (int64_t)p * n;
    // the job's diagonal 64 x 64 blocks (int8), zeroed before the rows fill them
    uint8_t *dq = dblk ? dblk + (size_t)dboff[q] * DBLK_BYTES : nullptr;
    if (dq) {
        const int n16 = qb_tile_ms(m) * DBLK_BYTES / 16;
        for (int t = tid; t < n16; t += 256) reinterpret_cast<uint4 *>(dq)[t] = make_uint4(0, 0, 0, 0);
    }
    for (int a = tid; a < m; a += 256) {
        const int j = idx[base + a];
        S[a] = j;
        ys[a] = X[xo + j];
    }
    __syncthreads();
    uint32_t *tile = tiles + (int64_t)base * W;
    for (int a = tid; a < m; a += 256) {
        const int i = S[a];
        const int32_t qii = diag[i];
        const int32_t f0 = qii + 2 * (H[xo + i] - qii * (int32_t)ys[a]);
        F0[base + a] = f0;
        y0[base + a] = ys[a];
        const uint32_t *row = ell + (int64_t)i * W;
        uint32_t *out = tile + (int64_t)a * W;
        const int cnt = ecnt[i];
        int k = 0;
        int32_t rowsum = 0;
        for (int t = 0; t < cnt; ++t) {
            const uint32_t w = row[t];
            const int col = qb_ell_col(w);
            int lo = 0, hi = m - 1, pos = -1;
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                const int sm = S[mid];
                if (sm == col) {
                    pos = mid;
                    break;
                }
                if (sm < col)
                    lo = mid + 1;
                else
                    hi = mid - 1;
            }
            if (pos >= 0) {
                const int32_t v = qb_ell_val(w);
                out[k++] = qb_ell_word(v, pos);
                rowsum += v * (int32_t)ys[pos];
                // column a & 63 of the block holds T[b][a] for the rows b of a's block
                if (dq && (pos >> 6) == (a >> 6))
                    dq[(size_t)(a >> 6) * DBLK_BYTES + (a & 63) * 64 + (pos & 63)] = (uint8_t)(int8_t)v;
            }
        }
        for (; k < W; ++k) out[k] = 0u;
        if (c) c[base + a] = f0 - 2 * rowsum;
    }
}

// ------------------------------------------------------------------ anneal
template <int MS>
__global__ void __launch_bounds__(1024) k_anneal_ell(const int32_t *__restrict__ jobs, int rgroups,
                                                     const int32_t *__restrict__ off, int W,
                                                     const uint32_t *__restrict__ tiles,
                                                     const int32_t *__restrict__ F0,
                                                     const uint8_t *__restrict__ y0, int nsw, int B,
                                                     const int32_t *__restrict__ thr, int R, int rw, uint32_t k0,
                                                     uint32_t k1, uint32_t inst_base, const qb_iter *__restrict__ it, uint8_t *__restrict__ Y,
                                                     int64_t *__restrict__ eout, int32_t *__restrict__ acnt)
{
    constexpr int MP = 64 * MS;
    extern __shared__ __align__(16) uint32_t dl[];
    const int q = jobs[blockIdx.x / rgroups];
    const int rg = blockIdx.x % rgroups;
    const int base = off[q], m = off[q + 1] - base;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int r = rg * rw + wid;

    uint32_t *tl = dl;                                   // [m][W]
    int32_t *F = reinterpret_cast<int32_t *>(dl + (size_t)MP * W) + wid * MP;
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(tiles + (int64_t)base * W);
        uint4 *dst = reinterpret_cast<uint4 *>(tl);
        const int n16 = m * W / 4;
        for (int t = tid; t < n16; t += blockDim.x) dst[t] = src[t];
    }
#pragma unroll
    for (int s = 0; s < MS; ++s) {
        const int pos = 64 * s + lane;
        F[pos] = pos < m ? F0[base + pos] : 0;
    }
    __syncthreads();
    if (r >= R) return;   // no barrier follows

    uint32_t ybits = 0;
    uint64_t active[MS];
#pragma unroll
    for (int s = 0; s < MS; ++s) {
        const int pos = 64 * s + lane;
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
            const uint4 o = qb_philox(make_uint4(((uint32_t)g << 6) | (uint32_t)lane, (uint32_t)sw, (uint32_t)r, tag),
                                      k0, k1);
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
            if (pend == 0) continue;
            int32_t fs = F[64 * s + lane];
            // the first 64 words of the row of lane kp, read one accept ahead:
            // kp is the next accepting lane of the current ballot, which is
            // most often the next accept, and its row read then overlaps the
            // current update instead of following it
            int kp = -1;
            uint32_t wp = 0u;
            while (true) {
                const uint32_t yb = (ybits >> s) & 1u;
                const int32_t dE = yb ? -fs : fs;
                const uint64_t acc = __ballot(dE <= tv[s]) & pend;
                if (acc == 0) break;
                const int k = __builtin_ctzll(acc);
                const int32_t dEk = __builtin_amdgcn_readlane(dE, k);
                const int32_t ykb = __builtin_amdgcn_readlane((int32_t)yb, k);
                e += dEk;
                ++nacc;
                const int32_t d2 = ykb ? -2 : 2;
                if (lane == k) ybits ^= 1u << s;
                const uint32_t *row = tl + (size_t)(64 * s + k) * W;
                // (word lane of a row is inside the LDS allocation for every
                // lane: the fields of the replicas follow the tile)
                uint32_t w0 = wp;
                if (kp != k) w0 = row[lane];
                if (lane < W && w0 != 0u) atomicAdd(&F[qb_ell_col(w0)], d2 * qb_ell_val(w0));
                for (int t0 = 64; t0 < W; t0 += 64) {
                    if (t0 + lane < W) {
                        const uint32_t wd = row[t0 + lane];
                        if (wd != 0u) atomicAdd(&F[qb_ell_col(wd)], d2 * qb_ell_val(wd));
                    }
                }
                // issued after the adds (which return nothing), so only the
                // read of the fields below waits for it
                const uint64_t rest = acc & ~((2ull << k) - 1ull);
                kp = rest ? __builtin_ctzll(rest) : -1;
                if (kp >= 0) wp = tl[(size_t)(64 * s + kp) * W + lane];
                pend &= ~((2ull << k) - 1ull);
                fs = F[64 * s + lane];
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
    if (acnt && lane == 0) acnt[(size_t)q * R + r] = nacc;
}

// The same sweep with the block's own couplings in registers (int8 tiles,
// W <= 64).  Lane L holds column L of the current diagonal block, T[64 s +
// k][64 s + L] for k < 64 (written by the extraction), so an accept moves
// the block's move values dE = sigma F by a register read -- the dense
// owner's accept chain, with no LDS access on it.  The F of every position
// still lives in LDS and still receives every entry of each accepted row by
// an LDS atomic add, so it is exact at the start of each block; those adds
// are issued one accept late (the row read overlaps the next accept's
// chain) and are never read back within the block.  A lane that flips has
// its sigma negated, but its dE is not read again in the block and the
// negation commutes with the later updates (the dense kernel's argument).
// The next block's column is loaded a whole block ahead, into the other of
// two register sets (even and odd blocks).
__device__ __forceinline__ int32_t dcol_at(const uint32_t (&d)[16], int k)
{
    // v_bfe_i32 takes its offset modulo 32 (bits [4:0]), so 8 k selects
    // byte k & 3 without a mask
    return __builtin_amdgcn_sbfe((int)d[k >> 2], (uint32_t)k * 8u, 8u);
}

__device__ __forceinline__ void load_dcol(uint32_t (&d)[16], const uint8_t *__restrict__ src)
{
    const uint4 *v = reinterpret_cast<const uint4 *>(src);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint4 t = v[i];
        d[4 * i + 0] = t.x;
        d[4 * i + 1] = t.y;
        d[4 * i + 2] = t.z;
        d[4 * i + 3] = t.w;
    }
}

template <int MS>
__global__ void __launch_bounds__(512) k_anneal_ell_dc(const int32_t *__restrict__ jobs, int rgroups,
                                                        const int32_t *__restrict__ off, int W,
                                                        const uint32_t *__restrict__ tiles,
                                                        const uint8_t *__restrict__ dblk,
                                                        const int32_t *__restrict__ dboff,
                                                        const int32_t *__restrict__ F0,
                                                        const uint8_t *__restrict__ y0, int nsw, int B,
                                                        const int32_t *__restrict__ thr, int R, int rw, uint32_t k0,
                                                        uint32_t k1, uint32_t inst_base,
                                                        const qb_iter *__restrict__ it, uint8_t *__restrict__ Y,
                                                        int64_t *__restrict__ eout, int32_t *__restrict__ acnt)
{
    constexpr int MP = 64 * MS;
    extern __shared__ __align__(16) uint32_t dl[];
    const int q = jobs[blockIdx.x / rgroups];
    const int rg = blockIdx.x % rgroups;
    const int base = off[q], m = off[q + 1] - base;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int r = rg * rw + wid;

    // Per wave MP fields and then 64 dump words: dump word L (F[MP + L])
    // holds the ELL word (column MP + L, value 0) and only ever receives
    // zeros.  A padding word at position w of a staged row becomes that same
    // word for column MP + w, so every lane adds its row word without a
    // branch or mask: a padding word, or a lane past the row reading its own
    // dump word, adds zero into its own dump word (no two lanes share one).
    uint32_t *tl = dl;                                   // [m][W]
    int32_t *F = reinterpret_cast<int32_t *>(dl + (size_t)MP * W) + wid * (MP + 64);
    {
        const uint32_t *src = tiles + (int64_t)base * W;
        const int nw = m * W;
        for (int t = tid; t < nw; t += blockDim.x) {
            const uint32_t v = src[t];
            tl[t] = v != 0u ? v : (uint32_t)(MP + t % W);
        }
    }
#pragma unroll
    for (int s = 0; s < MS; ++s) {
        const int pos = 64 * s + lane;
        F[pos] = pos < m ? F0[base + pos] : 0;
    }
    F[MP + lane] = MP + lane;
    __syncthreads();
    if (r >= R) return;   // no barrier follows

    const uint8_t *dq = dblk + (size_t)dboff[q] * DBLK_BYTES + lane * 64;
    // byte offset of a row word in LDS: row_offset * rsel + rbase, with rsel =
    // 1 and rbase = 4 L for a lane L < W, else rsel = 0 and rbase the lane's
    // dump word (row offsets stay below 1024 * 64 * 4 < 2^24, the range of
    // the 24-bit multiply)
    uint32_t rsel = lane < W ? 1u : 0u;
    asm volatile("" : "+v"(rsel));   // opaque: one multiply-add, not a select
    const uint32_t rbase = lane < W ? 4u * (uint32_t)lane
                                    : (uint32_t)(reinterpret_cast<const char *>(F + MP + lane) -
                                                 reinterpret_cast<const char *>(dl));
    uint32_t ybits = 0;
#pragma unroll
    for (int s = 0; s < MS; ++s) {
        const int pos = 64 * s + lane;
        if (pos < m && y0[base + pos]) ybits |= 1u << s;
    }
    int64_t e = 0;
    int32_t nacc = 0;
    const uint32_t tag = (1u << 28) | (inst_base + (it ? it->inst : 0u) + (uint32_t)q);
    constexpr int G = (MS + 3) / 4;
    const int sh = 32 - B;
    const int nblk = (m + 63) >> 6;                      // blocks with positions
    // the columns of the even and of the odd blocks: once block s is done,
    // its set is refilled with block s + 2 (in sweep order), a whole block
    // ahead of its use.  An odd block count is padded with one block without
    // positions, so that a block's parity, and with it its set, is the same
    // in every sweep.  With one block the column never changes.
    uint32_t cA[16], cB[16];
    const int nbe = nblk + (nblk & 1);
    load_dcol(cA, dq);
    if (MS > 1 && nblk > 1) load_dcol(cB, dq + DBLK_BYTES);
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
    // F of the next block, read as soon as the block before it has issued
    // its last add (every earlier atomic add of this wave precedes the read,
    // so it is exact), so that its latency overlaps that block's bookkeeping
    int32_t fsn = F[lane];

    for (int sw = 0; sw < nsw; ++sw) {
        int32_t tv[MS];
#pragma unroll
        for (int s = 0; s < MS; ++s) tv[s] = tvn[s];
        if (sw + 1 < nsw) thresholds(sw + 1, tvn);
#pragma unroll
        for (int s = 0; s < MS; ++s) {
            if (s < nblk) {
            const int na = min(m - 64 * s, 64);
            const uint32_t(&dc)[16] = (s & 1) ? cB : cA;
            const int32_t fs = fsn;
            const int32_t M0 = ((ybits >> s) & 1u) ? -1 : 0;
            const int32_t s2 = M0 ? -2 : 2, ns2 = -s2;   // 2 sigma
            int32_t dE = (fs ^ M0) - M0;
            // y of the block's lanes at its start: a lane accepts at most once
            // in the block, so an accepted lane's y is still this bit
            const uint64_t ym0 = __ballot(M0 != 0);
            uint64_t amask = 0;        // lanes accepted in the block
            int32_t eb = 0;            // their dE: at most 64 moves of |dE| < 2^24
            // the lane's threshold while it may still accept in the block: a
            // lane past the block, or at or below the last accept, gets
            // INT32_MIN, which no dE reaches (|dE| < 2^24), so the ballot
            // needs no mask of pending lanes
            int32_t tk = lane < na ? tv[s] : INT32_MIN;
            uint64_t acc = __ballot(dE <= tk);
            // the previous accept's row word and factor (a lane's own dump
            // word before the first accept); its adds are issued one accept
            // late, so the read is not waited for on the accept chain
            uint32_t pwr = (uint32_t)(MP + lane);
            int32_t pd2 = 0;
            while (acc) {
                const int k = __builtin_ctzll(acc);
                const uint64_t bk = 1ull << k;
                eb += __builtin_amdgcn_readlane(dE, k);
                amask |= bk;
                int32_t f, d2, yk;
                qb_accept_sign<false>(ym0, k, s2, ns2, f, d2, yk);
                dE += __mul24(f, dcol_at(dc, k));
                tk = lane <= k ? INT32_MIN : tk;
                const uint64_t accn = __ballot(dE <= tk);
                // the chain of this accept is done: only now wait for the
                // previous accept's row word and add it, then read this one's
                __builtin_amdgcn_sched_barrier(0);
                atomicAdd(&F[qb_ell_col(pwr)], __mul24(pd2, qb_ell_val(pwr)));
                // row word of lane L < W, else the lane's dump word
                pwr = *reinterpret_cast<const uint32_t *>(
                    reinterpret_cast<const char *>(dl) +
                    __umul24((uint32_t)((64 * s + k) * W * 4), rsel) + rbase);
                pd2 = d2;
                acc = accn;
            }
            atomicAdd(&F[qb_ell_col(pwr)], __mul24(pd2, qb_ell_val(pwr)));
            fsn = F[64 * (s + 1 < nblk ? s + 1 : 0) + lane];
            e += eb;
            nacc += __builtin_popcountll(amask);
            const uint32_t yb = (uint32_t)((ym0 ^ amask) >> lane) & 1u;
            ybits = (ybits & ~(1u << s)) | (yb << s);
            }
            if (MS > 1 && s < nbe) {
                int t = s + 2;
                if (t >= nbe) t -= nbe;
                if (t < nblk) load_dcol((s & 1) ? cB : cA, dq + (size_t)t * DBLK_BYTES);
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
    if (acnt && lane == 0) acnt[(size_t)q * R + r] = nacc;
}

constexpr size_t LDS_MAX = 160 * 1024;

// The job's ELL tile, each replica's fields, and 64 words per replica (the
// register-block kernel's dump area).
inline size_t ell_lds_bytes(int ms, int W, int rw)
{
    return sizeof(uint32_t) * ((size_t)64 * ms * (W + rw) + (size_t)64 * rw);
}

template <int MS>
qb_status launch_ell(int njobs, int rw, int R, hipStream_t s, const int32_t *jobs, qb_batch b, int W,
                     const uint32_t *tiles, const int32_t *F0, const uint8_t *y0, int nsw, int B, const int32_t *thr,
                     uint64_t seed, uint32_t inst_base, const qb_iter *it, uint8_t *Y, int64_t *e)
{
    const size_t lds = ell_lds_bytes(MS, W, rw);
    if (b->dblk_valid && W <= 64 && rw <= 8) {
        // the extraction wrote the int8 diagonal blocks after the ELL rows
        // (at most 8 replicas per workgroup: up to 256 registers per lane
        // hold the two column sets; beyond, the in-LDS kernel, same result)
        QB_TRY_HIP(hipFuncSetAttribute((const void *)k_anneal_ell_dc<MS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)LDS_MAX));
        const int rgroups = (R + rw - 1) / rw;
        const uint8_t *dblk = reinterpret_cast<const uint8_t *>(tiles + (int64_t)b->total * W);
        k_anneal_ell_dc<MS><<<njobs * rgroups, 64 * rw, lds, s>>>(jobs, rgroups, b->off_d, W, tiles, dblk, b->dboff_d,
                                                                  F0, y0, nsw, B, thr, R, rw, (uint32_t)seed,
                                                                  (uint32_t)(seed >> 32), inst_base, it, Y, e,
                                                                  b->acnt_d);
        QB_LAUNCH_CHECK();
        return QB_OK;
    }
    // set on every launch (no cached flag shared between devices or threads)
    QB_TRY_HIP(hipFuncSetAttribute((const void *)k_anneal_ell<MS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)LDS_MAX));
    const int rgroups = (R + rw - 1) / rw;
    k_anneal_ell<MS><<<njobs * rgroups, 64 * rw, lds, s>>>(jobs, rgroups, b->off_d, W, tiles, F0, y0, nsw, B, thr, R,
                                                           rw, (uint32_t)seed, (uint32_t)(seed >> 32), inst_base, it,
                                                           Y, e, b->acnt_d);
    QB_LAUNCH_CHECK();
    return QB_OK;
}

qb_status dispatch_ell(int cls, int njobs, int rw, int R, hipStream_t s, const int32_t *jobs, qb_batch b, int W,
                       const uint32_t *tiles, const int32_t *F0, const uint8_t *y0, int nsw, int B,
                       const int32_t *thr, uint64_t seed, uint32_t inst_base, const qb_iter *it, uint8_t *Y, int64_t *e)
{
#define QB_ARGS njobs, rw, R, s, jobs, b, W, tiles, F0, y0, nsw, B, thr, seed, inst_base, it, Y, e
    switch (cls) {
    case 0: return launch_ell<16>(QB_ARGS);
    case 1: return launch_ell<8>(QB_ARGS);
    case 2: return launch_ell<4>(QB_ARGS);
    case 3: return launch_ell<2>(QB_ARGS);
    case 4: return launch_ell<1>(QB_ARGS);
    }
#undef QB_ARGS
    return QB_E_UNSUPPORTED;
}

}  // namespace

extern "C" qb_status qb_extract_ell(qb_problem P, qb_batch b, const uint8_t *X_d, const int32_t *H_d,
                                   uint32_t *tile_d, int32_t *c_d, int32_t *F0_d, uint8_t *y0_d, void *stream)
{
    if (!P || !b || !X_d || !H_d || !tile_d || !F0_d || !y0_d) return QB_E_ARG;
    if (b->n != P->n) return QB_E_ARG;
    if (!P->sparse) return QB_E_UNSUPPORTED;
    if ((uintptr_t)tile_d & 15) return QB_E_ARG;
    if (b->J == 0) return QB_OK;
    // int8 problems also get the jobs' diagonal blocks (for the annealer's register path)
    uint8_t *dblk = P->int8_ok ? reinterpret_cast<uint8_t *>(tile_d + (int64_t)b->total * P->ellw) : nullptr;
    k_extract_ell<<<b->J, 256, 0, qb_stream(stream)>>>(P->ell, P->ellw, P->ecnt, P->diag, P->n, b->sol_d, b->off_d,
                                                       b->idx_d, X_d, H_d, tile_d, c_d, F0_d, y0_d, dblk, b->dboff_d);
    b->dblk_valid = dblk != nullptr;
    QB_LAUNCH_CHECK();
    return QB_OK;
}

qb_status qb_anneal_ell_x(qb_batch b, int32_t W, const uint32_t *tile_d, const int32_t *F0_d, const uint8_t *y0_d,
                          int32_t nsw, int32_t B, const int32_t *thr_d, int32_t R, int32_t rw, uint64_t seed,
                          uint32_t inst_base, const qb_iter *it, uint8_t *Y_d, int64_t *e_d, void *stream)
{
    if (!b || !tile_d || !F0_d || !y0_d || !thr_d || !Y_d || !e_d) return QB_E_ARG;
    if (nsw < 1 || B < 1 || B > 16 || R < 1 || R > 16 || rw < 0 || rw > 16) return QB_E_ARG;
    if (W < 4 || (W & 3) || W > 65536) return QB_E_ARG;
    if ((uintptr_t)tile_d & 15) return QB_E_ARG;
    if ((uint64_t)inst_base + (uint64_t)b->J > (1ull << 28)) return QB_E_RANGE;
    hipStream_t s = qb_stream(stream);
    // every size class starts at once: the fork precedes the first launch
    int ncls = 0;
    for (int c = 0; c < QB_NCLASS; ++c) ncls += b->cls_end[c] > b->cls_begin[c];
    if (ncls > 1) QB_TRY_HIP(hipEventRecord(b->ev_fork, s));
    bool first = true;
    for (int c = 0; c < QB_NCLASS; ++c) {
        const int nj = b->cls_end[c] - b->cls_begin[c];
        if (nj <= 0) continue;
        const int ms = qb_ms_of_class(c);
        int r2 = rw;
        if (r2 == 0) {
            // automatic: up to 8 replicas per workgroup, fewer when LDS is short
            r2 = R < 8 ? R : 8;
            while (r2 > 1 && ell_lds_bytes(ms, W, r2) > LDS_MAX) r2 >>= 1;
        }
        if (ell_lds_bytes(ms, W, r2) > LDS_MAX) return QB_E_CAPACITY;
        hipStream_t ls = s;
        if (!first) {
            ls = b->side[c];
            QB_TRY_HIP(hipStreamWaitEvent(ls, b->ev_fork, 0));
        }
        const qb_status rc = dispatch_ell(c, nj, r2, R, ls, b->lpt_d + b->cls_begin[c], b, W, tile_d, F0_d, y0_d, nsw,
                                          B, thr_d, seed, inst_base, it, Y_d, e_d);
        if (rc != QB_OK) return rc;
        if (!first) {
            QB_TRY_HIP(hipEventRecord(b->ev_join[c], ls));
            QB_TRY_HIP(hipStreamWaitEvent(s, b->ev_join[c], 0));
        }
        first = false;
    }
    return QB_OK;
}

extern "C" qb_status qb_anneal_ell(qb_batch b, int32_t W, const uint32_t *tile_d, const int32_t *F0_d,
                                  const uint8_t *y0_d, int32_t nsw, int32_t B, const int32_t *thr_d, int32_t R,
                                  int32_t rw, uint64_t seed, uint32_t inst_base, uint8_t *Y_d, int64_t *e_d,
                                  void *stream)
{
    return qb_anneal_ell_x(b, W, tile_d, F0_d, y0_d, nsw, B, thr_d, R, rw, seed, inst_base, nullptr, Y_d, e_d, stream);
}
