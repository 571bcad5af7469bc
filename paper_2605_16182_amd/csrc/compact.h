// Two-pass stream compaction for wave64 CDNA.
//
// The items [0, n) are split in tiles of CT_TILE; wavefront w of a tile's
// workgroup owns the tile's items [w * CT_WAVE, (w + 1) * CT_WAVE), 64 per
// round. Pass one counts the flagged items of every tile (one ballot per
// round, nothing written per item); the tile counts are scanned; pass two
// evaluates the flags again and calls op.emit(i, k) for the k-th flagged item
// i (k counted over [0, n) in index order). Neither pass writes a per-item
// flag or rank array, which the flags -> scan -> scatter form reads and
// writes several times over.
//
// An Op provides
//   static constexpr bool kHoist;    // evaluate every round's flag first
//   __device__ bool flag(int64_t i) const;                  // i < n
// With kHoist, flag is also evaluated (and its result dropped) at i = n - 1
// for the lanes past the end, so that every round's loads issue
// unconditionally and stay in flight together: flag must then read only
// inside [0, n) without branching around its loads. (This pays for 4-byte
// flag inputs; with 8-byte ones the rounds already keep the memory busy.)
//   __device__ void emit(int64_t i, uint32_t k) const;      // flagged i
//   __device__ void end(int64_t n, uint32_t total) const;   // once, after all
// end() runs in pass two on the lane holding item n - 1.
#pragma once

#include "tw_internal.h"

namespace tw {

constexpr int CT_THREADS = 256;
constexpr int CT_ROUNDS = 16;
constexpr int CT_WAVE = 64 * CT_ROUNDS;
constexpr int CT_TILE = (CT_THREADS / 64) * CT_WAVE;
static_assert(CT_TILE == GS_TILE, "staged group counts use the compaction's tiles");

template <class Op>
__global__ void __launch_bounds__(CT_THREADS)
k_ct_count(const Op op, int64_t n, uint32_t* __restrict__ cnt) {
    __shared__ uint32_t wsum[CT_THREADS / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t wb = (int64_t)tile * CT_TILE + (int64_t)wave * CT_WAVE;
    uint32_t c = 0;
    if constexpr (Op::kHoist) {
        bool f[CT_ROUNDS];
#pragma unroll
        for (int r = 0; r < CT_ROUNDS; ++r) {
            const int64_t i = wb + r * 64 + lane;
            f[r] = op.flag(i < n ? i : n - 1) && i < n;
        }
#pragma unroll
        for (int r = 0; r < CT_ROUNDS; ++r) c += (uint32_t)__popcll(__ballot(f[r]));
    } else {
        for (int r = 0; r < CT_ROUNDS; ++r) {
            const int64_t i = wb + r * 64 + lane;
            c += (uint32_t)__popcll(__ballot(i < n && op.flag(i)));
        }
    }
    if (lane == 0) wsum[wave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
#pragma unroll
        for (int w = 0; w < CT_THREADS / 64; ++w) t += wsum[w];
        cnt[tile] = t;
    }
}

template <class Op>
__global__ void __launch_bounds__(CT_THREADS)
k_ct_emit(const Op op, int64_t n, const uint32_t* __restrict__ off) {
    __shared__ uint32_t wsum[CT_THREADS / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t wb = (int64_t)tile * CT_TILE + (int64_t)wave * CT_WAVE;
    const uint64_t lower = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    uint32_t bits = 0, c = 0;  // this lane's flags (bit r: round r); the wave's count
    if constexpr (Op::kHoist) {
#pragma unroll
        for (int r = 0; r < CT_ROUNDS; ++r) {
            const int64_t i = wb + r * 64 + lane;
            bits |= (uint32_t)(op.flag(i < n ? i : n - 1) && i < n) << r;
        }
#pragma unroll
        for (int r = 0; r < CT_ROUNDS; ++r) c += (uint32_t)__popcll(__ballot((bits >> r) & 1u));
    } else {
        for (int r = 0; r < CT_ROUNDS; ++r) {
            const int64_t i = wb + r * 64 + lane;
            const bool f = i < n && op.flag(i);
            bits |= (uint32_t)f << r;
            c += (uint32_t)__popcll(__ballot(f));
        }
    }
    if (lane == 0) wsum[wave] = c;
    __syncthreads();
    uint32_t run = off[tile];
    for (int w = 0; w < wave; ++w) run += wsum[w];
    for (int r = 0; r < CT_ROUNDS; ++r) {
        const int64_t i = wb + r * 64 + lane;
        const bool f = (bits >> r) & 1u;
        const uint64_t b = __ballot(f);
        const uint32_t k = run + (uint32_t)__popcll(b & lower);
        if (f) op.emit(i, k);
        if (i == n - 1) op.end(n, k + (f ? 1u : 0u));
        run += (uint32_t)__popcll(b);
    }
}

// Runs both passes on stream s; *total (device) receives the flagged count.
// tiles holds the tile counts (grown as needed). counted: the caller already
// wrote every tile's count of flagged items into tiles (a producer that read
// the flags' inputs anyway), so the counting pass is skipped.
template <class Op>
hipError_t compact(const Op& op, int64_t n, uint32_t* total, DevBuf& tiles, Workspace& ws,
                   hipStream_t s, bool counted = false) {
    if (n <= 0) return scan_exclusive_u32(nullptr, nullptr, 0, total, ws, s);
    const int64_t nb = ceil_div(n, (int64_t)CT_TILE);
    hipError_t e = ensure(tiles, sizeof(uint32_t) * (nb + 1), s);
    if (e != hipSuccess) return e;
    uint32_t* cnt = tiles.as<uint32_t>();
    if (!counted)
        hipLaunchKernelGGL(k_ct_count<Op>, dim3((unsigned)nb), dim3(CT_THREADS), 0, s, op, n,
                           cnt);
    if ((e = scan_exclusive_u32(cnt, cnt, nb, total, ws, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_ct_emit<Op>, dim3((unsigned)nb), dim3(CT_THREADS), 0, s, op, n, cnt);
    return hipGetLastError();
}

}  // namespace tw
