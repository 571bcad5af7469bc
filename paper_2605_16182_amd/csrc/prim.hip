// Data-parallel primitives for the index rebuild, written for wave64 CDNA:
// an exclusive scan and a stable LSD radix sort whose per-tile ranks come
// from wave ballots (each lane learns which lanes of its wavefront share its
// digit from one ballot per digit bit, then counts the lower ones).
#include <algorithm>
#include <type_traits>

#include "compact.h"
#include "tw_internal.h"

namespace tw {

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

constexpr int RS_THREADS = 256;
constexpr int RS_WAVES = RS_THREADS / 64;
// keys per thread of a radix tile: 16 (4096-key tiles) for large sorts, 8
// for sorts of up to RS_SMALL keys (twice the workgroups, fewer registers:
// 8 % faster on 10M source ids, 6 % slower on 100M)
constexpr int RS_ITEMS = 16;
constexpr int RS_ITEMS_SMALL = 8;
constexpr int64_t RS_SMALL = 1 << 24;

template <typename V>
__device__ inline V wave_incl_scan(V v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        V o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    return v;
}

// exclusive scan of one value per thread over a 256-thread block; returns
// this thread's exclusive prefix and writes the block total to *total
template <typename V>
__device__ inline V block_excl_scan(V v, V* total) {
    __shared__ V wsum[SCAN_THREADS / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    V inc = wave_incl_scan(v);
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    V before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < SCAN_THREADS / 64; ++w) {
        V s = wsum[w];
        before += (w < wave) ? s : 0;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

// In is the input element type, widened to V for the sums
template <typename In, typename V>
__global__ void k_scan_reduce(const In* __restrict__ in, int64_t n, V* __restrict__ part) {
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    V s = 0;
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int64_t i = base + (int64_t)j * SCAN_THREADS + threadIdx.x;
        if (i < n) s += (V)in[i];
    }
    V total;
    block_excl_scan(s, &total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// one block: exclusive scan of the partials in place, total to *total
template <typename V>
__global__ void k_scan_partials(V* part, int64_t nb, V* total) {
    __shared__ V carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += SCAN_THREADS) {
        int64_t i = base + threadIdx.x;
        V v = i < nb ? part[i] : 0;
        V tot;
        V ex = block_excl_scan(v, &tot);
        V c = carry;
        if (i < nb) part[i] = c + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry = c + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

// sum of part[0, b) over the block (every thread gets it)
template <typename V>
__device__ inline V block_prefix_of(const V* __restrict__ part, int64_t b) {
    V p = 0;
    for (int64_t i = threadIdx.x; i < b; i += SCAN_THREADS) p += part[i];
    V all;
    block_excl_scan(p, &all);
    return all;
}

// SUM: the block's prefix is summed from the raw partials of the blocks
// before it (one launch fewer; for at most SCAN_SUM_MAX_BLOCKS blocks, whose
// partials stay in L2), and the last block writes the total (nullable);
// otherwise part holds the scanned partials.
constexpr int64_t SCAN_SUM_MAX_BLOCKS = 4096;

template <typename In, typename V, bool SUM>
__global__ void k_scan_down(const In* in, V* out, int64_t n, const V* __restrict__ part,
                            V* total) {
    __shared__ V tile[SCAN_TILE];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int k = j * SCAN_THREADS + threadIdx.x;
        int64_t i = base + k;
        tile[k] = i < n ? (V)in[i] : 0;
    }
    __syncthreads();
    V loc[SCAN_ITEMS];
    V s = 0;
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        loc[j] = s;
        s += tile[threadIdx.x * SCAN_ITEMS + j];
    }
    V tot;
    const V ex = block_excl_scan(s, &tot);
    const V bp = SUM ? block_prefix_of(part, blockIdx.x) : part[blockIdx.x];
    const V pre = ex + bp;
    if (SUM && total && threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) *total = bp + tot;
    for (int j = 0; j < SCAN_ITEMS; ++j) tile[threadIdx.x * SCAN_ITEMS + j] = pre + loc[j];
    __syncthreads();
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int k = j * SCAN_THREADS + threadIdx.x;
        int64_t i = base + k;
        if (i < n) out[i] = tile[k];
    }
}

template <typename V>
__global__ void k_set(V* p, V v) { *p = v; }

// Four u32 scans at once (array blockIdx.y of the launch): the same steps
// as above, one launch each instead of one per array.
struct Scan4 {
    const uint32_t* in[4];
    uint32_t* out[4];
    uint32_t* total[4];
};

// the element count of a scan: n, or, with n_dev, n_dev[0] + n_dev[1]
// (counted on the device) capped at n
__device__ inline int64_t scan_count(int64_t n, const uint32_t* n_dev) {
    if (!n_dev) return n;
    const int64_t c = (int64_t)n_dev[0] + (int64_t)n_dev[1];
    return c < n ? c : n;
}

__global__ void k_scan4_reduce(const Scan4 a, int64_t cap, uint32_t* __restrict__ part,
                               int64_t nb, const uint32_t* n_dev) {
    const int64_t n = scan_count(cap, n_dev);
    const int y = blockIdx.y;
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    uint32_t s = 0;
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int64_t i = base + (int64_t)j * SCAN_THREADS + threadIdx.x;
        if (i < n) s += a.in[y][i];
    }
    uint32_t total;
    block_excl_scan(s, &total);
    if (threadIdx.x == 0) part[y * nb + blockIdx.x] = total;
}

__global__ void k_scan4_partials(const Scan4 a, uint32_t* part, int64_t nb) {
    const int y = blockIdx.x;
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += SCAN_THREADS) {
        int64_t i = base + threadIdx.x;
        uint32_t v = i < nb ? part[y * nb + i] : 0;
        uint32_t tot;
        uint32_t ex = block_excl_scan(v, &tot);
        uint32_t c = carry;
        if (i < nb) part[y * nb + i] = c + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry = c + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && a.total[y]) *a.total[y] = carry;
}

template <bool SUM>
__global__ void k_scan4_down(const Scan4 a, int64_t cap, const uint32_t* __restrict__ part,
                             int64_t nb, const uint32_t* n_dev) {
    const int64_t n = scan_count(cap, n_dev);
    __shared__ uint32_t tile[SCAN_TILE];
    const int y = blockIdx.y;
    const uint32_t* in = a.in[y];
    uint32_t* out = a.out[y];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int k = j * SCAN_THREADS + threadIdx.x;
        int64_t i = base + k;
        tile[k] = i < n ? in[i] : 0;
    }
    __syncthreads();
    uint32_t loc[SCAN_ITEMS];
    uint32_t s = 0;
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        loc[j] = s;
        s += tile[threadIdx.x * SCAN_ITEMS + j];
    }
    uint32_t tot;
    const uint32_t ex = block_excl_scan(s, &tot);
    const uint32_t bp =
        SUM ? block_prefix_of(part + y * nb, blockIdx.x) : part[y * nb + blockIdx.x];
    const uint32_t pre = ex + bp;
    if (SUM && a.total[y] && threadIdx.x == 0 && blockIdx.x == gridDim.x - 1)
        *a.total[y] = bp + tot;
    for (int j = 0; j < SCAN_ITEMS; ++j) tile[threadIdx.x * SCAN_ITEMS + j] = pre + loc[j];
    __syncthreads();
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int k = j * SCAN_THREADS + threadIdx.x;
        int64_t i = base + k;
        if (i < n) out[i] = tile[k];
    }
}


// group starts of a timestamp sequence (group_starts)
struct GroupStartOp {
    const int64_t* ts;
    int has_last;
    int64_t last_ts;
    uint32_t pos_base;
    uint32_t* g_off;
    static constexpr bool kHoist = false;
    __device__ bool flag(int64_t i) const {
        return i == 0 ? (!has_last || ts[0] != last_ts) : ts[i] != ts[i - 1];
    }
    __device__ void emit(int64_t i, uint32_t k) const { g_off[k] = pos_base + (uint32_t)i; }
    __device__ void end(int64_t n, uint32_t total) const { g_off[total] = pos_base + (uint32_t)n; }
};

// ------------------------------------------------------------ radix sort
//
// A tile is RS_THREADS * ITEMS consecutive items; wavefront w of its
// workgroup owns the tile's items [w * WAVE_ITEMS, (w + 1) * WAVE_ITEMS),
// 64 per round.
// Ranks are wavefront-private (no workgroup barrier per round): in each round
// the lanes sharing a digit learn each other from one ballot per digit bit,
// and the lowest of them advances the wavefront's count for that digit. (LDS
// atomics in the histogram pass measured slower on source-id keys, whose
// skew makes many lanes of a wavefront hit one counter.)

// Digits of up to 8 bits (256 digits, one per thread of the workgroup) or,
// for sorts whose key bits take one pass fewer that way, up to 9 bits (512
// digits, two per thread: 2 tid and 2 tid + 1).
template <int RADIX>
struct Digits {
    static_assert(RADIX == RS_THREADS || RADIX == 2 * RS_THREADS, "one or two digits a thread");
    static constexpr int PER = RADIX / RS_THREADS;
    static constexpr int BITS = RADIX == 512 ? 9 : 8;
};

// lanes of the wavefront whose digit (of nbits <= MAXB bits) equals this
// lane's, among valid lanes: one ballot per digit bit; a lane collects the
// lanes whose bit differs from its own and keeps the others
template <int MAXB>
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid, int nbits) {
    const uint64_t live = __ballot(valid);
    uint64_t differ = 0;
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        if (b < nbits) {
            // all ones when the bit is set (a signed one-bit field extract)
            const uint32_t m = (uint32_t)((int32_t)(d << (31 - b)) >> 31);
            const uint64_t bal = __ballot(m != 0u);
            differ |= bal ^ (((uint64_t)m << 32) | m);
        }
    }
    return live & ~differ;
}

template <typename K, int ITEMS, int RADIX>
__global__ void __launch_bounds__(RS_THREADS)
k_rs_hist(const K* __restrict__ keys, int64_t n, int shift, int nbits,
          uint32_t* __restrict__ hist, int64_t nblocks) {
    using D = Digits<RADIX>;
    constexpr int TILE = RS_THREADS * ITEMS, WAVE_ITEMS = TILE / RS_WAVES;
    __shared__ uint32_t cnt[RS_WAVES][RADIX];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int w = 0; w < RS_WAVES; ++w)
#pragma unroll
        for (int q = 0; q < D::PER; ++q) cnt[w][tid * D::PER + q] = 0;
    __syncthreads();
    const uint32_t mask = (1u << nbits) - 1u;
    const uint64_t lower = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint32_t tile = xcd_tile(blockIdx.x, (uint32_t)nblocks);
    const int64_t wbase = (int64_t)tile * TILE + (int64_t)wave * WAVE_ITEMS;
    K k[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const int64_t i = wbase + r * 64 + lane;
        k[r] = i < n ? keys[i] : K(0);
    }
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const bool valid = wbase + r * 64 + lane < n;
        const uint32_t d = (uint32_t)(k[r] >> shift) & mask;
        const uint64_t peers = digit_peers<D::BITS>(d, valid, nbits);
        if (valid && (peers & lower) == 0) cnt[wave][d] += (uint32_t)__popcll(peers);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < D::PER; ++q) {
        const int d = tid * D::PER + q;
        uint32_t c = 0;
#pragma unroll
        for (int w = 0; w < RS_WAVES; ++w) c += cnt[w][d];
        hist[(int64_t)d * nblocks + tile] = c;
    }
}

// Scatter one tile to its stable output slots. offs[d * nblocks + b] is the
// first output slot of digit d for tile b (exclusive scan of the histogram).
// The tile is first ordered by digit in LDS, one array at a time, so that
// consecutive lanes write consecutive slots of each digit's run.
// W64: the items carry a 64-bit payload (v64); without it the LDS staging
// area is as wide as the widest of key and 32-bit value. PACK (with W64):
// the 32-bit value and the 64-bit payload (a timestamp) are read and leave
// packed as one 64-bit payload, (v64 - pack_base) << 32 | val.
template <typename K, bool W64, bool PACK, int ITEMS, int RADIX>
__global__ void __launch_bounds__(RS_THREADS)
k_rs_scatter(const K* __restrict__ keys, const uint32_t* __restrict__ vals,
             const uint64_t* __restrict__ v64, int64_t n, int shift, int nbits,
             const uint32_t* __restrict__ offs, int64_t nblocks, K* __restrict__ keys_out,
             uint32_t* __restrict__ vals_out, uint64_t* __restrict__ v64_out, uint64_t pack_base) {
    static_assert(W64 || !PACK, "packing needs the 64-bit payload");
    using D = Digits<RADIX>;
    constexpr int TILE = RS_THREADS * ITEMS, WAVE_ITEMS = TILE / RS_WAVES;
    using Stage = std::conditional_t<W64 || sizeof(K) == 8, uint64_t, uint32_t>;
    __shared__ uint32_t cnt[RS_WAVES][RADIX];  // wave counts, then wave starts
    __shared__ uint32_t lstart[RADIX];         // tile-local first slot of each digit
    __shared__ uint32_t gstart[RADIX];         // output slot of that first item
    __shared__ Stage stage[TILE];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t mask = (1u << nbits) - 1u;
    const uint64_t lower = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint32_t tile = xcd_tile(blockIdx.x, (uint32_t)nblocks);
#pragma unroll
    for (int q = 0; q < D::PER; ++q) {
        const int d = tid * D::PER + q;
#pragma unroll
        for (int w = 0; w < RS_WAVES; ++w) cnt[w][d] = 0;
        gstart[d] = offs[(int64_t)d * nblocks + tile];
    }
    __syncthreads();
    const int64_t tile0 = (int64_t)tile * TILE;
    const int64_t wbase = tile0 + (int64_t)wave * WAVE_ITEMS;
    const int tile_n = (int)std::min<int64_t>(TILE, n - tile0);

    // every input of the tile is loaded up front
    K k[ITEMS];
    uint32_t lp[ITEMS], v[ITEMS];
    uint64_t w2[W64 ? ITEMS : 1];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const int64_t i = wbase + r * 64 + lane;
        k[r] = i < n ? keys[i] : K(0);
        v[r] = (vals && i < n) ? vals[i] : 0u;
        if constexpr (PACK) w2[r] = i < n ? ((v64[i] - pack_base) << 32) | v[r] : 0ull;
        else if constexpr (W64) w2[r] = i < n ? v64[i] : 0ull;
    }

    // stable rank of each item among the wavefront's items of its digit
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const bool valid = wbase + r * 64 + lane < n;
        const uint32_t d = (uint32_t)(k[r] >> shift) & mask;
        const uint64_t peers = digit_peers<D::BITS>(d, valid, nbits);
        const uint32_t before = cnt[wave][d];
        lp[r] = before + (uint32_t)__popcll(peers & lower);
        if (valid && (peers & lower) == 0) cnt[wave][d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();

    // digit starts in the tile (scan over digits), then each wavefront's start
    uint32_t wpre[D::PER][RS_WAVES], tot[D::PER], sum = 0;
#pragma unroll
    for (int q = 0; q < D::PER; ++q) {
        tot[q] = 0;
#pragma unroll
        for (int w = 0; w < RS_WAVES; ++w) {
            wpre[q][w] = tot[q];
            tot[q] += cnt[w][tid * D::PER + q];
        }
        sum += tot[q];
    }
    uint32_t all;
    uint32_t ls = block_excl_scan<uint32_t>(sum, &all);
#pragma unroll
    for (int q = 0; q < D::PER; ++q) {
        const int d = tid * D::PER + q;
        lstart[d] = ls;
#pragma unroll
        for (int w = 0; w < RS_WAVES; ++w) cnt[w][d] = ls + wpre[q][w];
        ls += tot[q];
    }
    __syncthreads();

    // keys: into LDS in digit order, then out; each thread keeps the output
    // slots of the LDS slots it wrote out for the value arrays
    K* sk = reinterpret_cast<K*>(stage);
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        if (wbase + r * 64 + lane < n) {
            const uint32_t d = (uint32_t)(k[r] >> shift) & mask;
            lp[r] += cnt[wave][d];
            sk[lp[r]] = k[r];
        }
    }
    __syncthreads();
    uint32_t gp[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const int sl = r * RS_THREADS + tid;
        gp[r] = 0;
        if (sl < tile_n) {
            const K key = sk[sl];
            const uint32_t d = (uint32_t)(key >> shift) & mask;
            gp[r] = gstart[d] + ((uint32_t)sl - lstart[d]);
            keys_out[gp[r]] = key;
        }
    }
    if (!PACK && vals) {
        __syncthreads();
        uint32_t* sv = reinterpret_cast<uint32_t*>(stage);
#pragma unroll
        for (int r = 0; r < ITEMS; ++r)
            if (wbase + r * 64 + lane < n) sv[lp[r]] = v[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            const int sl = r * RS_THREADS + tid;
            if (sl < tile_n) vals_out[gp[r]] = sv[sl];
        }
    }
    if constexpr (W64) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < ITEMS; ++r)
            if (wbase + r * 64 + lane < n) stage[lp[r]] = w2[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            const int sl = r * RS_THREADS + tid;
            if (sl < tile_n) v64_out[gp[r]] = stage[sl];
        }
    }
}

// keys copied and (val, v64) packed as in k_rs_scatter<.., PACK>, for sorts
// with no pass to do it
template <typename K>
__global__ void k_pack_payload(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                               const uint64_t* __restrict__ win, int64_t n, uint64_t base,
                               K* __restrict__ kout, uint64_t* __restrict__ wout) {
    const int64_t i = (int64_t)blockIdx.x * SCAN_THREADS + threadIdx.x;
    if (i >= n) return;
    kout[i] = kin[i];
    wout[i] = ((win[i] - base) << 32) | vin[i];
}

// Sort (kin, vin, win) into (kout, vout, wout). Inputs are only read; when
// they alias the outputs the sort works in place. Passes alternate between
// the outputs and the workspace buffers, arranged so that the last pass
// lands in the outputs (a final copy happens only for an in-place sort with
// an odd number of passes).
template <typename K>
hipError_t radix_sort_impl(const K* kin0, const uint32_t* vin0, const uint64_t* win0, K* kout,
                           uint32_t* vout, uint64_t* wout, int64_t n, int bit_lo, int bit_hi,
                           Workspace& ws, hipStream_t s, bool pack = false,
                           uint64_t pack_base = 0) {
    hipError_t e;
    const bool has_v = vout != nullptr, has_w = wout != nullptr;
    if (pack && (bit_hi <= bit_lo || n <= 1)) {
        if (n <= 0) return hipSuccess;
        hipLaunchKernelGGL((k_pack_payload<K>), dim3((unsigned)ceil_div(n, (int64_t)SCAN_THREADS)),
                           dim3(SCAN_THREADS), 0, s, kin0, vin0, win0, n, pack_base, kout, wout);
        return hipGetLastError();
    }
    if (bit_hi <= bit_lo || n <= 1) {
        if (n > 0 && kin0 != kout) {
            if ((e = hipMemcpyAsync(kout, kin0, sizeof(K) * n, hipMemcpyDeviceToDevice, s)))
                return e;
            if (has_v && (e = hipMemcpyAsync(vout, vin0, 4 * n, hipMemcpyDeviceToDevice, s)))
                return e;
            if (has_w && (e = hipMemcpyAsync(wout, win0, 8 * n, hipMemcpyDeviceToDevice, s)))
                return e;
        }
        return hipSuccess;
    }
    // 9-bit digits where they save a pass (26-bit node ids: 3 passes, not 4)
    const bool wide = ceil_div(bit_hi - bit_lo, 9) < ceil_div(bit_hi - bit_lo, 8);
    const int passes = (int)ceil_div(bit_hi - bit_lo, wide ? 9 : 8);
    const bool in_place = (const void*)kin0 == (const void*)kout;
    if ((e = ensure(ws.keys_alt, sizeof(K) * n, s)) != hipSuccess) return e;
    if (has_v && (e = ensure(ws.vals_alt, sizeof(uint32_t) * n, s)) != hipSuccess) return e;
    if (has_w && (e = ensure(ws.v64_alt, sizeof(uint64_t) * n, s)) != hipSuccess) return e;
    K* ka = ws.keys_alt.as<K>();
    uint32_t* va = has_v ? ws.vals_alt.as<uint32_t>() : nullptr;
    uint64_t* wa = has_w ? ws.v64_alt.as<uint64_t>() : nullptr;
    // destination of pass p (0-based): the outputs when (passes - 1 - p) is
    // even, else the alternates; an in-place sort must start in the alternates
    const bool copy_back = in_place && (passes % 2 == 1);
    auto run = [&](auto items, auto radix) -> hipError_t {
        constexpr int I = decltype(items)::value;
        constexpr int R = decltype(radix)::value;
        const int64_t nblocks = ceil_div(n, (int64_t)RS_THREADS * I);
        hipError_t r = ensure(ws.hist, sizeof(uint32_t) * R * nblocks, s);
        if (r != hipSuccess) return r;
        uint32_t* hist = ws.hist.as<uint32_t>();
        const K* ki = kin0;
        const uint32_t* vi = vin0;
        const uint64_t* wi = win0;
        for (int p = 0; p < passes; ++p) {
            // the bits split evenly over the passes: fewer digits per pass
            // than 8 where that needs no extra pass (longer runs per digit)
            const int per = (bit_hi - bit_lo + passes - 1) / passes;
            const int sh = bit_lo + per * p;
            const int nb = bit_hi - sh < per ? bit_hi - sh : per;
            const bool to_out = copy_back ? (p % 2 == 1) : ((passes - 1 - p) % 2 == 0);
            K* ko = to_out ? kout : ka;
            uint32_t* vo = to_out ? vout : va;
            uint64_t* wo = to_out ? wout : wa;
            hipLaunchKernelGGL((k_rs_hist<K, I, R>), dim3(nblocks), dim3(RS_THREADS), 0, s, ki,
                               n, sh, nb, hist, nblocks);
            if ((r = scan_exclusive_u32(hist, hist, R * nblocks, nullptr, ws, s)) != hipSuccess)
                return r;
            if (pack && p == 0)
                hipLaunchKernelGGL((k_rs_scatter<K, true, true, I, R>), dim3(nblocks),
                                   dim3(RS_THREADS), 0, s, ki, vi, wi, n, sh, nb, hist, nblocks,
                                   ko, nullptr, wo, pack_base);
            else if (has_w)
                hipLaunchKernelGGL((k_rs_scatter<K, true, false, I, R>), dim3(nblocks),
                                   dim3(RS_THREADS), 0, s, ki, has_v ? vi : nullptr, wi, n, sh,
                                   nb, hist, nblocks, ko, vo, wo, 0ull);
            else
                hipLaunchKernelGGL((k_rs_scatter<K, false, false, I, R>), dim3(nblocks),
                                   dim3(RS_THREADS), 0, s, ki, has_v ? vi : nullptr, nullptr, n,
                                   sh, nb, hist, nblocks, ko, vo, nullptr, 0ull);
            ki = ko;
            vi = vo;
            wi = wo;
        }
        return hipSuccess;
    };
    using R8 = std::integral_constant<int, 256>;
    using R9 = std::integral_constant<int, 512>;
    using Small = std::integral_constant<int, RS_ITEMS_SMALL>;
    using Large = std::integral_constant<int, RS_ITEMS>;
    if (n <= RS_SMALL) e = wide ? run(Small{}, R9{}) : run(Small{}, R8{});
    else e = wide ? run(Large{}, R9{}) : run(Large{}, R8{});
    if (e != hipSuccess) return e;
    if (copy_back) {
        if ((e = hipMemcpyAsync(kout, ka, sizeof(K) * n, hipMemcpyDeviceToDevice, s))) return e;
        if (has_v && (e = hipMemcpyAsync(vout, va, 4 * n, hipMemcpyDeviceToDevice, s))) return e;
        if (has_w && (e = hipMemcpyAsync(wout, wa, 8 * n, hipMemcpyDeviceToDevice, s))) return e;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t ensure(DevBuf& b, size_t bytes, hipStream_t s) {
    if (bytes <= b.bytes) return hipSuccess;
    const size_t want = bytes + bytes / 4 + 256;
    // Stream-ordered growth: the new block is taken before the old one is
    // given back, so a failed growth leaves the buffer as it was, and the old
    // block returns to the pool only after the work already enqueued on s
    // (which may still read it) has run. Nothing waits on the host.
    void* p = nullptr;
    hipError_t e = hipMallocAsync(&p, want, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e;
    }
    if (b.p) {
        e = hipFreeAsync(b.p, s);
        if (e != hipSuccess) {
            (void)hipFreeAsync(p, s);
            return e;
        }
    }
    b.p = p;
    b.bytes = want;
    return hipSuccess;
}

void release(DevBuf& b, hipStream_t s) {
    if (b.p) (void)hipFreeAsync(b.p, s);
    b.p = nullptr;
    b.bytes = 0;
}

template <typename In, typename V>
hipError_t scan_core(const In* in, V* out, int64_t n, V* total, V* part, hipStream_t s) {
    if (n <= 0) {
        if (total) hipLaunchKernelGGL(k_set<V>, dim3(1), dim3(1), 0, s, total, (V)0);
        return hipGetLastError();
    }
    const int64_t nb = ceil_div(n, SCAN_TILE);
    hipLaunchKernelGGL((k_scan_reduce<In, V>), dim3(nb), dim3(SCAN_THREADS), 0, s, in, n, part);
    if (nb <= SCAN_SUM_MAX_BLOCKS) {
        hipLaunchKernelGGL((k_scan_down<In, V, true>), dim3(nb), dim3(SCAN_THREADS), 0, s, in,
                           out, n, part, total);
    } else {
        hipLaunchKernelGGL(k_scan_partials<V>, dim3(1), dim3(SCAN_THREADS), 0, s, part, nb, total);
        hipLaunchKernelGGL((k_scan_down<In, V, false>), dim3(nb), dim3(SCAN_THREADS), 0, s, in,
                           out, n, part, nullptr);
    }
    return hipGetLastError();
}

template <typename In, typename V>
hipError_t scan_exclusive(const In* in, V* out, int64_t n, V* total, DevBuf& part_buf,
                          hipStream_t s) {
    if (n > 0) {
        const hipError_t e = ensure(part_buf, sizeof(V) * (ceil_div(n, SCAN_TILE) + 1), s);
        if (e != hipSuccess) return e;
    }
    return scan_core<In, V>(in, out, n, total, part_buf.as<V>(), s);
}

hipError_t scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                              Workspace& ws, hipStream_t s) {
    return scan_exclusive<uint32_t, uint32_t>(in, out, n, total, ws.scan_part, s);
}

int64_t scan_parts_u32(int64_t n) { return ceil_div(std::max<int64_t>(n, 1), SCAN_TILE) + 1; }

hipError_t scan_exclusive_u32_into(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                                   uint32_t* part, hipStream_t s) {
    return scan_core<uint32_t, uint32_t>(in, out, n, total, part, s);
}

hipError_t scan_exclusive_u32x4(const uint32_t* const in[4], uint32_t* const out[4],
                                uint32_t* const total[4], int64_t n, Workspace& ws,
                                hipStream_t s, const uint32_t* n_dev) {
    Scan4 a;
    for (int y = 0; y < 4; ++y) {
        a.in[y] = in[y];
        a.out[y] = out[y];
        a.total[y] = total[y];
    }
    if (n <= 0) {
        for (int y = 0; y < 4; ++y)
            if (total[y]) hipLaunchKernelGGL(k_set<uint32_t>, dim3(1), dim3(1), 0, s, total[y], 0u);
        return hipGetLastError();
    }
    const int64_t nb = ceil_div(n, SCAN_TILE);
    hipError_t e = ensure(ws.scan_part, sizeof(uint32_t) * 4 * (nb + 1), s);
    if (e != hipSuccess) return e;
    uint32_t* part = ws.scan_part.as<uint32_t>();
    hipLaunchKernelGGL(k_scan4_reduce, dim3((unsigned)nb, 4), dim3(SCAN_THREADS), 0, s, a, n, part,
                       nb, n_dev);
    if (nb <= SCAN_SUM_MAX_BLOCKS) {
        hipLaunchKernelGGL(k_scan4_down<true>, dim3((unsigned)nb, 4), dim3(SCAN_THREADS), 0, s, a,
                           n, part, nb, n_dev);
    } else {
        hipLaunchKernelGGL(k_scan4_partials, dim3(4), dim3(SCAN_THREADS), 0, s, a, part, nb);
        hipLaunchKernelGGL(k_scan4_down<false>, dim3((unsigned)nb, 4), dim3(SCAN_THREADS), 0, s, a,
                           n, part, nb, n_dev);
    }
    return hipGetLastError();
}

hipError_t scan_exclusive_i32_to_u64(const int32_t* in, uint64_t* out, int64_t n, uint64_t* total,
                                     Workspace& ws, hipStream_t s) {
    return scan_exclusive<int32_t, uint64_t>(in, out, n, total, ws.scan_part, s);
}

hipError_t group_starts(int has_last, int64_t last_ts, const int64_t* ts, int64_t n,
                        uint32_t pos_base, uint32_t* g_off, uint32_t* total, Workspace& ws,
                        hipStream_t s, DevBuf* counted) {
    if (n <= 0) {
        hipLaunchKernelGGL(k_set<uint32_t>, dim3(1), dim3(1), 0, s, g_off, pos_base);
        hipLaunchKernelGGL(k_set<uint32_t>, dim3(1), dim3(1), 0, s, total, 0u);
        return hipGetLastError();
    }
    const GroupStartOp op{ts, has_last, last_ts, pos_base, g_off};
    if (counted) return compact(op, n, total, *counted, ws, s, true);
    return compact(op, n, total, ws.tiles, ws, s);
}

hipError_t radix_sort_u64(uint64_t* keys, uint32_t* vals, int64_t n, int bit_lo, int bit_hi,
                          Workspace& ws, hipStream_t s) {
    return radix_sort_impl<uint64_t>(keys, vals, nullptr, keys, vals, nullptr, n, bit_lo, bit_hi,
                                     ws, s);
}

hipError_t radix_sort_u32(uint32_t* keys, uint32_t* vals, int64_t n, int bit_lo, int bit_hi,
                          Workspace& ws, hipStream_t s) {
    return radix_sort_impl<uint32_t>(keys, vals, nullptr, keys, vals, nullptr, n, bit_lo, bit_hi,
                                     ws, s);
}

hipError_t radix_sort_u32_kv(const uint32_t* kin, const uint32_t* vin, const uint64_t* win,
                             uint32_t* kout, uint32_t* vout, uint64_t* wout, int64_t n, int bit_lo,
                             int bit_hi, Workspace& ws, hipStream_t s) {
    return radix_sort_impl<uint32_t>(kin, vin, win, kout, vout, wout, n, bit_lo, bit_hi, ws, s);
}

hipError_t radix_sort_u32_pack(const uint32_t* kin, const uint32_t* vin, const uint64_t* win,
                               uint64_t base, uint32_t* kout, uint64_t* pout, int64_t n,
                               int bit_lo, int bit_hi, Workspace& ws, hipStream_t s) {
    return radix_sort_impl<uint32_t>(kin, vin, win, kout, nullptr, pout, n, bit_lo, bit_hi, ws, s,
                                     true, base);
}

}  // namespace tw
