// The Ising-machine stage in Ising form (eq. 2, eq. 3): jobs given as
// couplings J (symmetric, zero diagonal), fields h and start spins s0 in
// {-1, +1} -- the native input of hardware Ising machines -- annealed on
// E'(s) = -sum_{a != b} J_ab s_a s_b - sum_a h_a s_a.
//
// Flipping spin k changes E' by 2 s_k g_k with the local field
// g_k = 2 sum_{b != k} J_kb s_b + h_k, and the flip moves every other field by
// -4 J_bk s_k.  Writing F = -2 g and y = (s + 1) / 2 this is exactly the
// QUBO sweep of the batched annealer with T = -4 J: the move is (1 - 2y_k) F_k
// (= 2 s_k g_k) and an accept adds 2 (1 - 2y_k) T_ik to F_i (= 8 J_ik s_k).
// So a prep kernel rewrites the job into that form (int16 tiles, F0, y0),
// the annealer runs unchanged, and a post kernel returns spins; thresholds
// are taken in E' units, energies come back in E' units.
#include <algorithm>

#include "qb_internal.h"

namespace {

constexpr int32_t JMAX = 8191;                 // |4 J| fits int16
constexpr int64_t GMAX = int64_t(1) << 30;     // |F| = 2 |g| fits int32

struct IsingWork {
    int16_t *tile;
    int32_t *F0;
    uint8_t *y0;
    uint8_t *Y;
    int32_t *bad;
};

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

IsingWork ising_layout(qb_batch b, int R, void *base, size_t *total)
{
    IsingWork w{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t t_o = take(sizeof(int16_t) * (size_t)std::max<int64_t>(b->tile_elems, 16));
    const size_t f_o = take(sizeof(int32_t) * (size_t)std::max(b->total, 1));
    const size_t y_o = take((size_t)std::max(b->total, 1));
    const size_t Y_o = take((size_t)std::max(b->total, 1) * R);
    const size_t b_o = take(sizeof(int32_t) * (size_t)std::max(b->J, 1));
    if (total) *total = off;
    char *p = (char *)base;
    if (p) {
        w.tile = (int16_t *)(p + t_o);
        w.F0 = (int32_t *)(p + f_o);
        w.y0 = (uint8_t *)(p + y_o);
        w.Y = (uint8_t *)(p + Y_o);
        w.bad = (int32_t *)(p + b_o);
    }
    return w;
}

// One workgroup per job, one wave per tile row: T = -4 J in the same layout,
// F0 = -2 g(s0), y0 = (s0 + 1) / 2, and a range flag for the job.
template <typename JT>
__global__ void __launch_bounds__(256) k_ising_prep(const int32_t *__restrict__ off,
                                                    const int64_t *__restrict__ tile_off,
                                                    const JT *__restrict__ Jt, const int32_t *__restrict__ h,
                                                    const int8_t *__restrict__ s0, int16_t *__restrict__ T16,
                                                    int32_t *__restrict__ F0, uint8_t *__restrict__ y0,
                                                    int32_t *__restrict__ bad)
{
    __shared__ int8_t ss[1024];
    __shared__ int32_t flag;
    const int q = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int base = off[q], m = off[q + 1] - base;
    const int MS = qb_tile_ms(m), MP = 64 * MS;
    if (tid == 0) flag = 0;
    __syncthreads();
    for (int a = tid; a < m; a += 256) {
        const int8_t v = s0[base + a];
        ss[a] = v;
        y0[base + a] = v > 0 ? 1 : 0;
        if (v != 1 && v != -1) atomicOr(&flag, 1);
    }
    __syncthreads();
    const JT *J = Jt + tile_off[q];
    int16_t *T = T16 + tile_off[q];
    for (int a = wid; a < MP; a += 4) {
        int64_t dot = 0;
        for (int s = 0; s < MS; ++s) {
            const int b = 64 * s + lane;
            const int64_t at = (int64_t)a * MP + lane * MS + s;
            int32_t v = 0;
            if (a < m && b < m && b != a) {
                v = (int32_t)J[at];
                // the mirror entry J[b][a] (the sweep reads rows as columns)
                if (v != (int32_t)J[(int64_t)b * MP + (a & 63) * MS + (a >> 6)]) atomicOr(&flag, 1);
            }
            if (v > JMAX || v < -JMAX) atomicOr(&flag, 1);
            T[at] = (int16_t)(-4 * max(min(v, JMAX), -JMAX));
            if (a < m && b < m) dot += (int64_t)v * ss[b];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) dot += __shfl_xor(dot, o, 64);
        if (lane == 0 && a < m) {
            const int64_t g = 2 * dot + h[base + a];
            if (g >= GMAX || g <= -GMAX) atomicOr(&flag, 1);
            const int64_t gc = g >= GMAX ? GMAX - 1 : g <= -GMAX ? -GMAX + 1 : g;
            F0[base + a] = (int32_t)(-2 * gc);
        }
    }
    __syncthreads();
    if (tid == 0) bad[q] = flag;
}

// Spins from the chosen states; a job with out-of-range input keeps s0 and
// reports e = INT64_MIN for every replica.
__global__ void __launch_bounds__(256) k_ising_post(int R, const int32_t *__restrict__ off,
                                                    const uint8_t *__restrict__ Y, const int8_t *__restrict__ s0,
                                                    const int32_t *__restrict__ bad, int8_t *__restrict__ S,
                                                    int64_t *__restrict__ e)
{
    const int q = blockIdx.x;
    const int base = off[q], m = off[q + 1] - base;
    const bool b = bad[q] != 0;
    for (int t = threadIdx.x; t < m * R; t += 256) {
        const int a = t % m;
        S[(int64_t)base * R + t] = b ? s0[base + a] : (Y[(int64_t)base * R + t] ? 1 : -1);
    }
    if (b)
        for (int r = threadIdx.x; r < R; r += 256) e[(int64_t)q * R + r] = INT64_MIN;
}

}  // namespace

extern "C" size_t qb_anneal_ising_workspace(qb_batch b, int32_t R)
{
    if (!b || R < 1) return 0;
    size_t total = 0;
    ising_layout(b, R, nullptr, &total);
    return total;
}

extern "C" qb_status qb_anneal_ising(qb_batch b, const void *J_tile_d, int32_t int8_tile, const int32_t *h_d,
                                    const int8_t *s0_d, int32_t nsw, int32_t B, const int32_t *thr_d, int32_t R,
                                    uint64_t seed, uint32_t inst_base, void *work_d, int8_t *S_d, int64_t *e_d,
                                    void *stream)
{
    if (!b || !J_tile_d || !h_d || !s0_d || !thr_d || !work_d || !S_d || !e_d) return QB_E_ARG;
    if (nsw < 1 || B < 1 || B > 16 || R < 1 || R > 16) return QB_E_ARG;
    if (((uintptr_t)J_tile_d & 15) || ((uintptr_t)work_d & 255)) return QB_E_ARG;
    if (b->J == 0) return QB_OK;
    hipStream_t s = qb_stream(stream);
    const IsingWork w = ising_layout(b, R, work_d, nullptr);
    if (int8_tile)
        k_ising_prep<int8_t><<<b->J, 256, 0, s>>>(b->off_d, b->tile_off_d, (const int8_t *)J_tile_d, h_d, s0_d,
                                                 w.tile, w.F0, w.y0, w.bad);
    else
        k_ising_prep<int16_t><<<b->J, 256, 0, s>>>(b->off_d, b->tile_off_d, (const int16_t *)J_tile_d, h_d, s0_d,
                                                  w.tile, w.F0, w.y0, w.bad);
    QB_LAUNCH_CHECK();
    qb_status rc = qb_anneal(b, w.tile, 0, w.F0, w.y0, nsw, B, thr_d, R, seed, inst_base, w.Y, e_d, stream);
    if (rc != QB_OK) return rc;
    k_ising_post<<<b->J, 256, 0, s>>>(R, b->off_d, w.Y, s0_d, w.bad, S_d, e_d);
    QB_LAUNCH_CHECK();
    return QB_OK;
}
