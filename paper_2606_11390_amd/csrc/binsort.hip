// Tile binning with a stable radix sort on the (tile id | depth) key (gfx950).
//
// Paper Section 4: per camera the Gaussians are sorted by depth before
// rasterisation, with one record per (Gaussian, tile) intersection; the paper
// uses a CUB radix sort.  The result here is the stable sort of the 64-bit
// key (global tile id << 32) | bits(depth) over intersections enumerated
// (view, Gaussian, tile row-major).
//
// An LSD radix sort processes the low (depth) digits first.  All intersections
// of one (view, Gaussian) pair share its depth, so the depth passes are run
// once per visible pair instead of once per intersection:
//   1. depth passes (4 x 8 bits) over the visible (view, Gaussian) pairs
//      (those with a non-empty tile rectangle), the first pass compacting
//      them out of the projection outputs;
//   2. the pairs' tile rectangles gathered into that order (by the last
//      depth pass, beside the pair indices it scatters: the only random
//      access of the binning after the sort) and an exclusive scan of their
//      tile counts;
//   3. load-balanced emission of (global tile id, Gaussian) pairs, each
//      pair's tiles in row-major order;
//   4. stable passes over the tile-id bits;
//   5. per-tile [start, end) ranges.
// Because every pass is stable, this equals the stable sort of the full key
// over the (view, Gaussian, tile) enumeration, equal keys in Gaussian order.
//
// Each pass is reduce-then-scan: per-block digit histograms, a per-digit scan
// across blocks, then a scatter that ranks keys stably inside 2048-key chunks
// (wave ballots match equal digits, wave-private LDS counters order waves)
// and writes them through LDS so that runs of equal digits leave coalesced.
// Every element count is read from device memory, so no call syncs the host.
#include "gs_device.h"

namespace gs {
namespace {

constexpr int RS_THREADS = 256;
constexpr int RS_WAVES = RS_THREADS / GS_WAVE;
constexpr int RS_ITEMS = 8;
constexpr int RS_CHUNK = RS_THREADS * RS_ITEMS;     // keys per chunk
constexpr int RS_WAVE_SPAN = GS_WAVE * RS_ITEMS;     // keys per wave per chunk
constexpr int RS_MAX_BLOCKS = 4096;
constexpr int RS_MAX_BITS = 9;    // widest digit: 512 counters per wave
constexpr int RS_RAW_MAX = 16;    // passes of at most this many blocks run without the per-digit scan kernel

enum Source { SRC_PAIRS = 0, SRC_PROJ = 1, SRC_TILE_LEN = 2, SRC_MORTON = 3 };

struct SortIO {
    const uint32_t* keys_in;   // SRC_PAIRS
    const uint32_t* vals_in;
    const float* depths;       // SRC_PROJ
    const int2* rects;
    const int2* ranges;        // SRC_TILE_LEN
    const float* means;        // SRC_MORTON: planar [3][n]
    float org[3], inv_cell[3];
    uint32_t* keys_out;
    uint32_t* vals_out;
    int2* rects_out;           // gathering scatter: rects[value] at each output position
    uint32_t n_const;          // element count when n_dev is NULL
    const uint32_t* n_dev;     // device element count
};

__device__ __forceinline__ uint32_t io_count(const SortIO& io)
{
    return io.n_dev ? *io.n_dev : io.n_const;
}

__device__ __forceinline__ void block_span(uint32_t n, int nb, int b, uint32_t& beg, uint32_t& end)
{
    uint32_t per = (n + (uint32_t)nb - 1u) / (uint32_t)nb;
    per = (per + RS_CHUNK - 1u) / RS_CHUNK * RS_CHUNK;
    const unsigned long long b0 = (unsigned long long)per * (unsigned)b;
    beg = (uint32_t)min((unsigned long long)n, b0);
    end = (uint32_t)min((unsigned long long)n, b0 + per);
}

// 10-bit cell of one coordinate: floor((x - org) * inv_cell) clamped to
// [0, 1023], float32 without contraction (a non-finite x lands in cell 0)
__device__ __forceinline__ uint32_t cell10(float x, float org, float inv)
{
#pragma clang fp contract(off)
    const float t = floorf((x - org) * inv);
    return t >= 1023.0f ? 1023u : (t >= 0.0f ? (uint32_t)t : 0u);
}

__device__ __forceinline__ uint32_t spread10(uint32_t x)
{
    // bit b of x moves to bit 3b
    x &= 0x3FFu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

// 30-bit Morton code: bit 3b + k holds bit b of axis k's cell (x: k = 0)
__device__ __forceinline__ uint32_t morton30(const float* __restrict__ means, uint32_t n, uint32_t i,
                                             const float* org, const float* inv)
{
    return spread10(cell10(means[i], org[0], inv[0])) | (spread10(cell10(means[n + i], org[1], inv[1])) << 1) |
           (spread10(cell10(means[2 * (size_t)n + i], org[2], inv[2])) << 2);
}

template <int SRC>
__device__ __forceinline__ bool load_kv(const SortIO& io, uint32_t i, uint32_t end, uint32_t& k,
                                        uint32_t& v)
{
    // the loads are unconditional, so that a caller's loads can all be in
    // flight at once: past the end (end >= 1 in every caller) they read the
    // last element, which is then reported invalid
    const bool in = i < end;
    const uint32_t j = in ? i : end - 1u;
    if (SRC == SRC_PAIRS) {
        k = io.keys_in[j];
        v = io.vals_in[j];
        return in;
    } else if (SRC == SRC_PROJ) {
        // a pair is binned when its tile rectangle is not empty
        const int2 rc = io.rects[j];
        k = __float_as_uint(io.depths[j]);
        v = i;
        const int w = (rc.y & 0xFFFF) - (rc.x & 0xFFFF), h = (int)((uint32_t)rc.y >> 16) - (int)((uint32_t)rc.x >> 16);
        return in && w > 0 && h > 0;
    } else if (SRC == SRC_MORTON) {
        k = morton30(io.means, io.n_const, j, io.org, io.inv_cell);
        v = i;
        return in;
    } else {
        // longest lists first: 255 minus the list length rounded down to four
        // significant bits (a one-pass key; the order only decides which
        // tiles start first)
        const int2 r = io.ranges[j];
        const uint32_t len = (uint32_t)min(max(r.y - r.x, 0), 0xFFFF);
        uint32_t code = len;
        if (len >= 8u) {
            const uint32_t e = 31u - (uint32_t)__clz(len);   // 3 .. 15
            code = ((e - 2u) << 3) | ((len >> (e - 3u)) & 7u);
        }
        k = 0xFFu - code;
        v = i;
        return in;
    }
}

// lanes of the wave holding the same digit as this lane.  NB is the widest
// digit the kernel instance handles; a narrower pass leaves the high bits of
// every digit zero, where all lanes agree, so the loop is unrolled to NB
// steps with no per-pass count.  Per bit: the lanes with the bit set (one
// ballot) and a mask that keeps them or their complement (xor, and).
template <int NB>
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid)
{
    const uint64_t v = __ballot(valid);
    uint32_t mlo = (uint32_t)v, mhi = (uint32_t)(v >> 32);
    const uint32_t dn = ~d;
#pragma unroll
    for (int k = 0; k < NB; k++) {
        // all ones where bit k of d is clear, zero where it is set
        const uint32_t nb = (uint32_t)((int)(dn << (31 - k)) >> 31);
        const uint64_t b = __ballot(nb == 0u);
        // m & (b ^ nb) in one gfx950 three-input logic op per half: with m as
        // the middle operand the function is symmetric in the outer two, so
        // table 0x48 (true for (1,1,0) and (0,1,1)) holds for either operand
        // order of the lookup index
        mlo = __builtin_amdgcn_bitop3_b32((uint32_t)b, mlo, nb, 0x48);
        mhi = __builtin_amdgcn_bitop3_b32((uint32_t)(b >> 32), mhi, nb, 0x48);
    }
    return valid ? (((uint64_t)mhi << 32) | mlo) : 0ull;
}

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const int l = __lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// exclusive scan of one uint32 per thread over a 256-thread block
__device__ __forceinline__ uint32_t block_excl_scan_256(uint32_t x, uint32_t* s_tmp, uint32_t& total)
{
    const int lane = __lane_id(), w = threadIdx.x / GS_WAVE;
    uint32_t inc = x;
    for (int o = 1; o < GS_WAVE; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == GS_WAVE - 1) s_tmp[w] = inc;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
    for (int i = 0; i < RS_WAVES; i++) {
        const uint32_t t = s_tmp[i];
        if (i < w) before += t;
        total += t;
    }
    __syncthreads();
    return before + inc - x;
}

// DBITS: the largest digit width a kernel instance handles (8 or 9 bits:
// 256 or 512 counters per wave in LDS); `bits` <= DBITS is the pass's width
template <int SRC, int DBITS>
__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(SortIO io, int shift, int bits,
                                                        uint32_t* __restrict__ hist)
{
    constexpr int ND = 1 << DBITS;
    __shared__ uint32_t s_cnt[RS_WAVES][ND];
    const int nb = gridDim.x, b = blockIdx.x, t = threadIdx.x, w = t / GS_WAVE;
    for (int i = t; i < RS_WAVES * ND; i += RS_THREADS) (&s_cnt[0][0])[i] = 0;
    __syncthreads();
    const uint32_t n = io_count(io);
    uint32_t beg, end;
    block_span(n, nb, b, beg, end);
    const uint32_t mask = (1u << bits) - 1u;
    const uint64_t lt = lanemask_lt();
    for (uint32_t base = beg; base < end; base += RS_CHUNK) {
        // all RS_ITEMS loads of a thread are issued before any is used
        uint32_t k[RS_ITEMS];
        bool valid[RS_ITEMS];
#pragma unroll
        for (int r = 0; r < RS_ITEMS; r++) {
            uint32_t v = 0;
            k[r] = 0;
            valid[r] = load_kv<SRC>(io, base + (uint32_t)(r * RS_THREADS + t), end, k[r], v);
        }
#pragma unroll
        for (int r = 0; r < RS_ITEMS; r++) {
            const uint32_t d = (k[r] >> shift) & mask;
            const uint64_t peers = match_digit<DBITS>(d, valid[r]);
            if (valid[r] && (peers & lt) == 0) s_cnt[w][d] += (uint32_t)__popcll(peers);
        }
    }
    __syncthreads();
    const int nd = 1 << bits;
    for (int d = t; d < nd; d += RS_THREADS) {
        uint32_t s = 0;
        for (int i = 0; i < RS_WAVES; i++) s += s_cnt[i][d];
        hist[(size_t)d * nb + b] = s;
    }
}

// one block per digit: exclusive scan of its counts across the nb blocks, in
// segments of blockDim.x counts with a running carry
__global__ __launch_bounds__(1024) void k_rs_spine(uint32_t* __restrict__ hist, int nb,
                                                   uint32_t* __restrict__ dtot)
{
    __shared__ uint32_t s_w[16];
    const int d = blockIdx.x, t = threadIdx.x, lane = __lane_id(), w = t / GS_WAVE;
    const int nw = blockDim.x / GS_WAVE;
    uint32_t carry = 0;
    for (int s0 = 0; s0 < nb; s0 += blockDim.x) {
        const int i = s0 + t;
        const uint32_t x = i < nb ? hist[(size_t)d * nb + i] : 0u;
        uint32_t inc = x;
        for (int o = 1; o < GS_WAVE; o <<= 1) {
            const uint32_t y = __shfl_up(inc, o);
            if (lane >= o) inc += y;
        }
        if (lane == GS_WAVE - 1) s_w[w] = inc;
        __syncthreads();
        uint32_t before = 0, total = 0;
        for (int k = 0; k < nw; k++) {
            if (k < w) before += s_w[k];
            total += s_w[k];
        }
        if (i < nb) hist[(size_t)d * nb + i] = carry + before + inc - x;
        carry += total;
        __syncthreads();
    }
    if (t == 0) dtot[d] = carry;
}

// exclusive scan over the ND digits of a 256-thread block, thread t owning
// digits t * DPT .. t * DPT + DPT - 1 (x: its DPT values, replaced by their
// exclusive prefixes); returns the total
template <int DPT>
__device__ __forceinline__ uint32_t block_excl_scan_digits(uint32_t (&x)[DPT], uint32_t* s_tmp)
{
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < DPT; i++) {
        const uint32_t v = x[i];
        x[i] = sum;
        sum += v;
    }
    uint32_t total;
    const uint32_t before = block_excl_scan_256(sum, s_tmp, total);
#pragma unroll
    for (int i = 0; i < DPT; i++) x[i] += before;
    return total;
}

// GATHER: the values are pair indices; each one's tile rectangle is read
// with it and written beside it (io.rects -> io.rects_out), so that the scan
// after the sort reads rectangles in order instead of gathering them
//
// raw: the per-digit scan across blocks was not run (a pass of at most
// RS_RAW_MAX blocks); excl then holds the histogram's counts and every block
// forms its own digit offsets and the digit totals from them.
template <int SRC, int DBITS, bool GATHER = false>
__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(SortIO io, int shift, int bits,
                                                           const uint32_t* __restrict__ excl,
                                                           const uint32_t* __restrict__ dtot,
                                                           uint32_t* __restrict__ count_out, int raw)
{
    constexpr int ND = 1 << DBITS;
    constexpr int DPT = ND / RS_THREADS;   // digits per thread in the digit scans
    static_assert(DPT >= 1 && ND % RS_THREADS == 0, "digit count");
    __shared__ uint32_t s_base[ND];
    __shared__ uint32_t s_wcnt[RS_WAVES][ND];
    __shared__ uint32_t s_cex[ND];
    __shared__ uint32_t s_tmp[RS_WAVES];
    __shared__ uint32_t s_k[RS_CHUNK];
    __shared__ uint32_t s_v[RS_CHUNK];
    __shared__ int2 s_r[GATHER ? RS_CHUNK : 1];
    const int nb = gridDim.x, b = blockIdx.x, t = threadIdx.x, w = t / GS_WAVE, lane = __lane_id();
    const int nd = 1 << bits;
    const uint32_t mask = (1u << bits) - 1u;

    const uint32_t n = io_count(io);
    uint32_t beg, end;
    block_span(n, nb, b, beg, end);
    const uint64_t lt = lanemask_lt();
    uint32_t key[RS_ITEMS], val[RS_ITEMS];
    bool ok[RS_ITEMS];
    // all loads of a thread for a chunk are issued before any is used; the
    // first chunk's are issued before the digit offsets below are set up, so
    // that both wait on memory together
    auto load_chunk = [&](uint32_t cb) {
        const uint32_t wb = cb + (uint32_t)w * RS_WAVE_SPAN;
#pragma unroll
        for (int r = 0; r < RS_ITEMS; r++) {
            key[r] = 0;
            val[r] = 0;
            ok[r] = load_kv<SRC>(io, wb + (uint32_t)(r * GS_WAVE + lane), end, key[r], val[r]);
        }
    };
    if (beg < end) load_chunk(beg);

    // global start of each digit for this block (the per-block offsets are
    // read with the digit totals, before the scan)
    {
        uint32_t x[DPT], ex[DPT];
        if (raw) {
            // a digit's counts over the nb <= RS_RAW_MAX blocks, sixteen loads
            // in flight at a time (unconditional, clamped to the last block)
#pragma unroll
            for (int i = 0; i < DPT; i++) {
                const int d = min(t * DPT + i, nd - 1);
                const uint32_t* row = excl + (size_t)d * nb;
                uint32_t tot = 0, before = 0;
                for (int b0 = 0; b0 < nb; b0 += 16) {
                    uint32_t h[16];
#pragma unroll
                    for (int u = 0; u < 16; u++) h[u] = row[min(b0 + u, nb - 1)];
#pragma unroll
                    for (int u = 0; u < 16; u++) {
                        const bool in = b0 + u < nb;
                        tot += in ? h[u] : 0u;
                        before += (in && b0 + u < b) ? h[u] : 0u;
                    }
                }
                x[i] = t * DPT + i < nd ? tot : 0u;
                ex[i] = t * DPT + i < nd ? before : 0u;
            }
        } else {
#pragma unroll
            for (int i = 0; i < DPT; i++) {
                const int d = t * DPT + i;
                x[i] = d < nd ? dtot[d] : 0u;
                ex[i] = d < nd ? excl[(size_t)d * nb + b] : 0u;
            }
        }
        const uint32_t all = block_excl_scan_digits<DPT>(x, s_tmp);
#pragma unroll
        for (int i = 0; i < DPT; i++) {
            const int d = t * DPT + i;
            s_base[d] = d < nd ? x[i] + ex[i] : 0u;
        }
        if (count_out && b == 0 && t == 0) *count_out = all;
    }

    for (uint32_t cb = beg; cb < end; cb += RS_CHUNK) {
        for (int i = t; i < RS_WAVES * nd; i += RS_THREADS) s_wcnt[i >> bits][i & (nd - 1)] = 0;
        __syncthreads();
        uint32_t rank[RS_ITEMS];
        int2 rct[GATHER ? RS_ITEMS : 1];
        if (cb != beg) load_chunk(cb);
        if (GATHER) {
            // every value is a pair index, also past the end (see load_kv)
#pragma unroll
            for (int r = 0; r < RS_ITEMS; r++) rct[r] = io.rects[val[r]];
        }
#pragma unroll
        for (int r = 0; r < RS_ITEMS; r++) {
            const uint32_t d = (key[r] >> shift) & mask;
            const uint64_t peers = match_digit<DBITS>(d, ok[r]);
            const uint32_t before = s_wcnt[w][d];
            rank[r] = before + (uint32_t)__popcll(peers & lt);
            if (ok[r] && (peers & lt) == 0) s_wcnt[w][d] = before + (uint32_t)__popcll(peers);
        }
        __syncthreads();
        // per digit: exclusive prefix across waves, chunk total, chunk digit start
        uint32_t tot[DPT];
#pragma unroll
        for (int i = 0; i < DPT; i++) {
            const int d = t * DPT + i;
            uint32_t acc = 0;
            if (d < nd) {
                for (int k = 0; k < RS_WAVES; k++) {
                    const uint32_t c = s_wcnt[k][d];
                    s_wcnt[k][d] = acc;
                    acc += c;
                }
            }
            tot[i] = acc;
        }
        uint32_t cex[DPT];
#pragma unroll
        for (int i = 0; i < DPT; i++) cex[i] = tot[i];
        const uint32_t ctot = block_excl_scan_digits<DPT>(cex, s_tmp);
#pragma unroll
        for (int i = 0; i < DPT; i++) s_cex[t * DPT + i] = cex[i];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RS_ITEMS; r++) {
            if (!ok[r]) continue;
            const uint32_t d = (key[r] >> shift) & mask;
            const uint32_t pos = s_cex[d] + s_wcnt[w][d] + rank[r];
            s_k[pos] = key[r];
            s_v[pos] = val[r];
            if (GATHER) s_r[pos] = rct[r];
        }
        __syncthreads();
        // write-out: a thread's RS_ITEMS slots j = t + r * RS_THREADS (the
        // chunk holds at most RS_CHUNK keys) are read from LDS together, then
        // their digits' offsets, so that the thread waits on LDS twice, not
        // twice per slot; slots at or past ctot hold stale keys whose masked
        // digits index the LDS arrays in range and are not written out
        uint32_t ko[RS_ITEMS], vo[RS_ITEMS], bo[RS_ITEMS], co[RS_ITEMS];
        int2 ro[GATHER ? RS_ITEMS : 1];
#pragma unroll
        for (int r = 0; r < RS_ITEMS; r++) {
            const uint32_t j = (uint32_t)(t + r * RS_THREADS);
            ko[r] = s_k[j];
            vo[r] = s_v[j];
            if (GATHER) ro[r] = s_r[j];
        }
#pragma unroll
        for (int r = 0; r < RS_ITEMS; r++) {
            const uint32_t d = (ko[r] >> shift) & mask;
            bo[r] = s_base[d];
            co[r] = s_cex[d];
        }
#pragma unroll
        for (int r = 0; r < RS_ITEMS; r++) {
            const uint32_t j = (uint32_t)(t + r * RS_THREADS);
            if (j >= ctot) continue;
            const uint32_t dst = bo[r] + j - co[r];
            if (io.keys_out) io.keys_out[dst] = ko[r];
            io.vals_out[dst] = vo[r];
            if (GATHER) io.rects_out[dst] = ro[r];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < DPT; i++) s_base[t * DPT + i] += tot[i];
    }
}

// ---------------------------------------------------------------------------
// tile rectangles in depth order, scan of their tile counts, intersection
// count, overflow
// ---------------------------------------------------------------------------
constexpr int SC_THREADS = 256;
constexpr int SC_ITEMS = 8;

// tiles of a packed rectangle (x0 | y0 << 16, x1 | y1 << 16); zero when empty
__device__ __forceinline__ uint32_t rect_count(int2 r)
{
    const int w = (r.y & 0xFFFF) - (r.x & 0xFFFF), h = (int)((uint32_t)r.y >> 16) - (int)((uint32_t)r.x >> 16);
    return (w > 0 && h > 0) ? (uint32_t)w * (uint32_t)h : 0u;
}

// exclusive scan of one uint64 per thread over a 256-thread block
__device__ __forceinline__ unsigned long long block_excl_scan_256_u64(unsigned long long x,
                                                                       unsigned long long* s_tmp,
                                                                       unsigned long long& total)
{
    const int lane = __lane_id(), w = threadIdx.x / GS_WAVE;
    unsigned long long inc = x;
    for (int o = 1; o < GS_WAVE; o <<= 1) {
        const unsigned long long y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == GS_WAVE - 1) s_tmp[w] = inc;
    __syncthreads();
    unsigned long long before = 0;
    total = 0;
    for (int i = 0; i < RS_WAVES; i++) {
        const unsigned long long t = s_tmp[i];
        if (i < w) before += t;
        total += t;
    }
    __syncthreads();
    return before + inc - x;
}

// sums the tile counts of the visible pairs' rectangles (in depth order, as
// the last depth pass wrote them) per block (64-bit: a pair may cover up to
// 2^32 - 1 tiles)
//
// It also zeroes the tile ranges (the range pass only writes non-empty tiles).
__global__ __launch_bounds__(SC_THREADS) void k_scan_reduce(const uint32_t* __restrict__ n_dev,
                                                            const int2* __restrict__ srect,
                                                            unsigned long long* __restrict__ part,
                                                            int2* __restrict__ ranges, long long n_ranges)
{
    __shared__ unsigned long long s_tmp[RS_WAVES];
    const int nb = gridDim.x, b = blockIdx.x, t = threadIdx.x;
    for (long long i = (long long)b * SC_THREADS + t; i < n_ranges; i += (long long)nb * SC_THREADS)
        ranges[i] = make_int2(0, 0);
    uint32_t beg, end;
    block_span(*n_dev, nb, b, beg, end);
    unsigned long long s = 0;
    for (uint32_t cb = beg; cb < end; cb += SC_THREADS * SC_ITEMS) {
        int2 rc[SC_ITEMS];
#pragma unroll
        for (int r = 0; r < SC_ITEMS; r++) {
            const uint32_t i = cb + (uint32_t)(r * SC_THREADS + t);
            rc[r] = i < end ? srect[i] : make_int2(0, 0);
        }
#pragma unroll
        for (int r = 0; r < SC_ITEMS; r++) s += rect_count(rc[r]);
    }
    unsigned long long tot;
    block_excl_scan_256_u64(s, s_tmp, tot);
    if (t == 0) part[b] = tot;
}

constexpr int EMIT_SPAN = 2048;   // output slots per emission workgroup

// sum of one uint64 per thread over a 256-thread block, returned to every thread
__device__ __forceinline__ unsigned long long block_sum_256_u64(unsigned long long x, unsigned long long* s_tmp)
{
    for (int o = GS_WAVE / 2; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if (__lane_id() == 0) s_tmp[threadIdx.x / GS_WAVE] = x;
    __syncthreads();
    unsigned long long total = 0;
    for (int i = 0; i < RS_WAVES; i++) total += s_tmp[i];
    __syncthreads();
    return total;
}

// Writes offs[i] (first output slot of source i, clamped to the capacity) and,
// for every emission workgroup k, bsrc[k] = the source whose slots contain
// slot k * EMIT_SPAN (each source has at least one slot, so exactly one does);
// bsrc[last] = the source holding the last emitted slot m - 1, where m is the
// intersection count clamped to the capacity.  Each block forms its own
// carry (the tile counts of the blocks before it) and the total from the
// nb per-block sums, so no separate scan of them runs; block 0 publishes the
// counts (cnt[1] = m, the info words).
__global__ __launch_bounds__(SC_THREADS) void k_scan_down(const int2* __restrict__ srect,
                                                          const unsigned long long* __restrict__ part,
                                                          uint32_t capacity, uint32_t* __restrict__ cnt,
                                                          int* __restrict__ info, uint32_t* __restrict__ offs,
                                                          uint32_t* __restrict__ bsrc, uint32_t last)
{
    __shared__ unsigned long long s_tmp[RS_WAVES];
    const int nb = gridDim.x, b = blockIdx.x, t = threadIdx.x;
    // the nb <= RS_MAX_BLOCKS block sums, a thread's loads all in flight at
    // once (unconditional, clamped to the last sum)
    constexpr int PER = RS_MAX_BLOCKS / SC_THREADS;
    unsigned long long xs[PER];
#pragma unroll
    for (int k = 0; k < PER; k++) xs[k] = part[min(t + k * SC_THREADS, nb - 1)];
    unsigned long long before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < PER; k++) {
        const int i = t + k * SC_THREADS;
        if (i < nb) {
            all += xs[k];
            if (i < b) before += xs[k];
        }
    }
    unsigned long long carry = block_sum_256_u64(before, s_tmp);
    const unsigned long long total = block_sum_256_u64(all, s_tmp);
    const unsigned long long cap = capacity;
    const unsigned long long m = total < cap ? total : cap;
    if (b == 0 && t == 0) {
        cnt[1] = (uint32_t)m;
        info[GS_INFO_VISIBLE] = (int)cnt[0];
        info[GS_INFO_ISECT] = (int)(total < 0x7FFFFFFFull ? total : 0x7FFFFFFFull);
        info[GS_INFO_OVERFLOW] = total > cap ? 1 : 0;
    }
    uint32_t beg, end;
    block_span(cnt[0], nb, b, beg, end);
    for (uint32_t cb = beg; cb < end; cb += SC_THREADS * SC_ITEMS) {
        // thread t owns SC_ITEMS consecutive elements
        uint32_t x[SC_ITEMS];
        unsigned long long s = 0;
        const uint32_t i0 = cb + (uint32_t)t * SC_ITEMS;
        // unconditional loads (clamped to the last element), all in flight at once
        int2 rc[SC_ITEMS];
#pragma unroll
        for (int r = 0; r < SC_ITEMS; r++) rc[r] = srect[min(i0 + (uint32_t)r, end - 1u)];
#pragma unroll
        for (int r = 0; r < SC_ITEMS; r++) {
            x[r] = i0 + r < end ? rect_count(rc[r]) : 0u;
            s += x[r];
        }
        unsigned long long tot;
        unsigned long long run = block_excl_scan_256_u64(s, s_tmp, tot);
        for (int r = 0; r < SC_ITEMS; r++) {
            const uint32_t i = i0 + r;
            if (i < end) {
                const unsigned long long o = carry + run;
                offs[i] = (uint32_t)(o < capacity ? o : capacity);
                // emission workgroups whose first slot lies in [o, o + x) below the capacity
                const unsigned long long lim = min(o + x[r], (unsigned long long)capacity);
                for (unsigned long long k = (o + EMIT_SPAN - 1) / EMIT_SPAN; k * EMIT_SPAN < lim; k++)
                    bsrc[k] = i;
                if (m > 0 && o <= m - 1 && m - 1 < o + x[r]) bsrc[last] = i;
            }
            run += x[r];
        }
        carry += tot;
    }
}

// ---------------------------------------------------------------------------
// load-balanced emission: one block per EMIT_SPAN consecutive output slots
// ---------------------------------------------------------------------------
constexpr int EMIT_THREADS = 256;

__global__ __launch_bounds__(EMIT_THREADS) void k_emit(const uint32_t* __restrict__ pids,
                                                       const uint32_t* __restrict__ offs,
                                                       const uint32_t* __restrict__ bsrc, uint32_t last,
                                                       const uint32_t* __restrict__ cnt,
                                                       const int2* __restrict__ srect, long long N,
                                                       ViewTable vt, uint32_t* __restrict__ keys_out,
                                                       uint32_t* __restrict__ vals_out, int hbits,
                                                       uint32_t* __restrict__ hist0)
{
    __shared__ uint32_t s_off[EMIT_SPAN + 1];
    __shared__ uint32_t s_gid[EMIT_SPAN + 1];
    __shared__ uint32_t s_base[EMIT_SPAN + 1];
    __shared__ uint32_t s_wt[EMIT_SPAN + 1];
    __shared__ uint32_t s_tx[EMIT_SPAN + 1];
    __shared__ __align__(16) uint32_t s_src[EMIT_SPAN];   // source of each slot
    __shared__ uint32_t s_wmax[EMIT_THREADS / GS_WAVE];
    __shared__ uint32_t s_h[1 << RS_MAX_BITS];
    // the views' tile-row widths and tile offsets, looked up per source (a
    // per-lane index into the argument block would be a vector load each)
    __shared__ int s_vtx[GS_MAX_VIEWS], s_vtoff[GS_MAX_VIEWS];
    const uint32_t m = cnt[1];
    const uint32_t start = blockIdx.x * (uint32_t)EMIT_SPAN;
    // with hist0: this workgroup's column of the first tile pass's digit
    // histogram (that pass then runs one EMIT_SPAN-slot chunk per block, so
    // block = workgroup)
    const int nd = hist0 ? 1 << hbits : 0;
    const size_t nbk = gridDim.x;
    for (int d = threadIdx.x; d < nd; d += EMIT_THREADS) s_h[d] = 0u;
    if (start >= m) {
        for (int d = threadIdx.x; d < nd; d += EMIT_THREADS) hist0[(size_t)d * nbk + blockIdx.x] = 0u;
        return;
    }
    const uint32_t end = min(m, start + (uint32_t)EMIT_SPAN);
    const int t = threadIdx.x, lane = __lane_id(), w = t / GS_WAVE;
    // sources of this workgroup's slots: from the one holding its first slot
    // to the one holding the next workgroup's first slot (which may start
    // exactly there; its slots then lie outside and are never selected)
    const uint32_t s0 = bsrc[blockIdx.x];
    const uint32_t s1 = end < m ? bsrc[blockIdx.x + 1] : bsrc[last];
    // at most EMIT_SPAN + 1 sources (each has at least one slot); the clamp
    // only guards the LDS arrays against inconsistent rectangles
    const uint32_t ns = min(s1 - s0 + 1, (uint32_t)EMIT_SPAN + 1);
    // every source's index, offset and rectangle are read in depth order
    // (consecutive), all loads of a thread issued before any is used
    constexpr int EMIT_SRC = (EMIT_SPAN + 1 + EMIT_THREADS - 1) / EMIT_THREADS;
    uint32_t pid[EMIT_SRC], off[EMIT_SRC];
    int2 rc[EMIT_SRC];
#pragma unroll
    for (int q = 0; q < EMIT_SRC; q++) {
        // unconditional loads (clamped to the last source, ns >= 1), all in flight at once
        const uint32_t k = min((uint32_t)(t + q * EMIT_THREADS), ns - 1u);
        pid[q] = pids[s0 + k];
        off[q] = offs[s0 + k];
        rc[q] = srect[s0 + k];
    }
    for (int i = t; i < EMIT_SPAN; i += EMIT_THREADS) s_src[i] = 0u;
    for (int i = t; i < vt.n_views; i += EMIT_THREADS) {
        s_vtx[i] = vt.tiles_x[i];
        s_vtoff[i] = vt.tile_off[i];
    }
    __syncthreads();
    // each source marks the slot where it starts (the first source, which
    // starts at or before this workgroup's first slot, marks slot 0); slots
    // of one source are consecutive and every source has one, so the source
    // of a slot is the last mark at or before it: a prefix maximum
#pragma unroll
    for (int q = 0; q < EMIT_SRC; q++) {
        const uint32_t k = (uint32_t)(t + q * EMIT_THREADS);
        if (k >= ns) continue;
        const uint32_t v = (uint32_t)(pid[q] / (unsigned long long)N);
        const uint32_t g = pid[q] - v * (uint32_t)N;
        const int x0 = rc[q].x & 0xFFFF, y0 = (int)((uint32_t)rc[q].x >> 16), x1 = rc[q].y & 0xFFFF;
        const int TX = s_vtx[v];
        s_off[k] = off[q];
        s_gid[k] = g;
        s_base[k] = (uint32_t)(s_vtoff[v] + y0 * TX + x0);
        s_wt[k] = (uint32_t)max(x1 - x0, 1);
        s_tx[k] = (uint32_t)TX;
        if (off[q] < end) s_src[off[q] > start ? off[q] - start : 0u] = k;
    }
    __syncthreads();
    // inclusive max-scan over the EMIT_SPAN marks, thread t owning 8 in a row
    static_assert(EMIT_SPAN == 8 * EMIT_THREADS, "8 slots per thread");
    uint4 a = *reinterpret_cast<const uint4*>(&s_src[8 * t]);
    uint4 b = *reinterpret_cast<const uint4*>(&s_src[8 * t + 4]);
    a.y = max(a.y, a.x); a.z = max(a.z, a.y); a.w = max(a.w, a.z);
    b.x = max(b.x, a.w); b.y = max(b.y, b.x); b.z = max(b.z, b.y); b.w = max(b.w, b.z);
    uint32_t inc = b.w;
    for (int o = 1; o < GS_WAVE; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o);
        if (lane >= o) inc = max(inc, y);
    }
    if (lane == GS_WAVE - 1) s_wmax[w] = inc;
    uint32_t ex = __shfl_up(inc, 1);
    if (lane == 0) ex = 0u;
    __syncthreads();
    for (int i = 0; i < w; i++) ex = max(ex, s_wmax[i]);
    a.x = max(a.x, ex); a.y = max(a.y, ex); a.z = max(a.z, ex); a.w = max(a.w, ex);
    b.x = max(b.x, ex); b.y = max(b.y, ex); b.z = max(b.z, ex); b.w = max(b.w, ex);
    *reinterpret_cast<uint4*>(&s_src[8 * t]) = a;
    *reinterpret_cast<uint4*>(&s_src[8 * t + 4]) = b;
    __syncthreads();
    const uint32_t hmask = (uint32_t)nd - 1u;
    for (uint32_t i = start + t; i < end; i += EMIT_THREADS) {
        const uint32_t lo = s_src[i - start];
        const uint32_t j = i - s_off[lo];
        const uint32_t wdt = s_wt[lo];
        const uint32_t row = j / wdt, col = j - row * wdt;
        const uint32_t key = s_base[lo] + row * s_tx[lo] + col;
        keys_out[i] = key;
        vals_out[i] = s_gid[lo];
        if (nd) atomicAdd(&s_h[key & hmask], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < nd; d += EMIT_THREADS) hist0[(size_t)d * nbk + blockIdx.x] = s_h[d];
}

// ---------------------------------------------------------------------------
// tile ranges
// ---------------------------------------------------------------------------
// 16-byte stores over the aligned body; the up to three elements before the
// first 16-byte boundary and after the last one are written singly
__global__ void k_fill_i32(int* __restrict__ p, int value, long long head, long long nv, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nv) reinterpret_cast<int4*>(p + head)[i] = make_int4(value, value, value, value);
    if (i < head) p[i] = value;
    const long long t0 = head + 4 * nv;
    if (i < n - t0) p[t0 + i] = value;
}

hipError_t fill_i32(int* p, int value, long long n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const long long head = min(n, (long long)(((16 - ((uintptr_t)p & 15)) & 15) / 4));
    const long long nv = (n - head) / 4;
    const long long threads = max(nv, 4ll);
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, p, value, head, nv, n);
    return hipGetLastError();
}

// thread t looks at keys 4t .. 4t + 3 (one 16-byte load) and their outer
// neighbours; a run boundary between two keys sets the end of one tile's
// range and the start of the next
__global__ void k_ranges(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ cnt,
                         uint32_t total_tiles, int2* __restrict__ ranges)
{
    const uint32_t m = cnt[1];
    const uint32_t i0 = 4u * (blockIdx.x * blockDim.x + threadIdx.x);
    if (i0 >= m) return;
    uint32_t k[6];   // keys i0 - 1 .. i0 + 4; 0xFFFFFFFF outside [0, m)
    k[0] = i0 > 0 ? keys[i0 - 1] : 0xFFFFFFFFu;
    if (i0 + 4 <= m) {
        const uint4 q = *reinterpret_cast<const uint4*>(keys + i0);
        k[1] = q.x; k[2] = q.y; k[3] = q.z; k[4] = q.w;
    } else {
        for (int r = 0; r < 4; r++) k[1 + r] = i0 + r < m ? keys[i0 + r] : 0xFFFFFFFFu;
    }
    k[5] = i0 + 4 < m ? keys[i0 + 4] : 0xFFFFFFFFu;
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const uint32_t i = i0 + r, c = k[1 + r];
        // keys >= total_tiles cannot occur for consistent inputs; never write out of range
        if (i >= m || c >= total_tiles) continue;
        if (k[r] != c) ranges[c].x = (int)i;
        if (k[r + 2] != c) ranges[c].y = (int)(i + 1);
    }
}

int sort_blocks(unsigned long long n_max)
{
    unsigned long long nb = (n_max + 2 * RS_CHUNK - 1) / (2 * RS_CHUNK);
    if (nb < 1) nb = 1;
    if (nb > RS_MAX_BLOCKS) nb = RS_MAX_BLOCKS;
    return (int)nb;
}

template <int SRC>
hipError_t radix_pass(const SortIO& io, int nb, int shift, int bits, uint32_t* hist, uint32_t* dtot,
                      uint32_t* count_out, hipStream_t st, bool have_hist = false)
{
    const int sp_threads = min(1024, ((nb + GS_WAVE - 1) / GS_WAVE) * GS_WAVE);
    // few blocks: each scatter block reads the counts of the blocks before it
    // (at most RS_RAW_MAX per digit) instead of a scan kernel's prefixes
    const int raw = nb <= RS_RAW_MAX ? 1 : 0;
    const bool gather = SRC == SRC_PAIRS && io.rects_out;
    if (bits <= 8) {
        if (!have_hist)
            hipLaunchKernelGGL((k_rs_hist<SRC, 8>), dim3(nb), dim3(RS_THREADS), 0, st, io, shift, bits, hist);
        if (!raw) hipLaunchKernelGGL(k_rs_spine, dim3(1u << bits), dim3(sp_threads), 0, st, hist, nb, dtot);
        if (gather)
            hipLaunchKernelGGL((k_rs_scatter<SRC, 8, true>), dim3(nb), dim3(RS_THREADS), 0, st, io, shift, bits,
                               hist, dtot, count_out, raw);
        else
            hipLaunchKernelGGL((k_rs_scatter<SRC, 8>), dim3(nb), dim3(RS_THREADS), 0, st, io, shift, bits, hist,
                               dtot, count_out, raw);
    } else {
        if (!have_hist)
            hipLaunchKernelGGL((k_rs_hist<SRC, RS_MAX_BITS>), dim3(nb), dim3(RS_THREADS), 0, st, io, shift, bits,
                               hist);
        if (!raw) hipLaunchKernelGGL(k_rs_spine, dim3(1u << bits), dim3(sp_threads), 0, st, hist, nb, dtot);
        if (gather)
            hipLaunchKernelGGL((k_rs_scatter<SRC, RS_MAX_BITS, true>), dim3(nb), dim3(RS_THREADS), 0, st, io, shift,
                               bits, hist, dtot, count_out, raw);
        else
            hipLaunchKernelGGL((k_rs_scatter<SRC, RS_MAX_BITS>), dim3(nb), dim3(RS_THREADS), 0, st, io, shift,
                               bits, hist, dtot, count_out, raw);
    }
    return hipGetLastError();
}

// widths of the fewest passes of at most RS_MAX_BITS bits covering `total`
// bits, split as evenly as possible (e.g. 32 -> 8, 8, 8, 8; 17 -> 9, 8)
int plan_passes(int total, int* widths)
{
    const int np = (total + RS_MAX_BITS - 1) / RS_MAX_BITS;
    for (int p = 0; p < np; p++) widths[p] = total / np + (p < total % np ? 1 : 0);
    return np;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// bsrc slot of the source holding the last emitted intersection (after the
// per-workgroup slots 0 .. ceil(cap / EMIT_SPAN) - 1)
uint32_t bsrc_last(unsigned long long cap) { return (uint32_t)((cap + EMIT_SPAN - 1) / EMIT_SPAN); }

struct BinWs {
    uint32_t *dk0, *dv0, *dk1, *dv1, *offs, *tk, *tv, *hist, *dtot, *cnt, *bsrc;
    unsigned long long* part;
    int2* srect;
    size_t bytes;
};

BinWs bin_layout(char* base, unsigned long long vn, unsigned long long cap)
{
    BinWs w;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char* p = base + o;
        o += align256(bytes);
        return p;
    };
    w.dk0 = (uint32_t*)take(4 * vn);
    w.dv0 = (uint32_t*)take(4 * vn);
    w.dk1 = (uint32_t*)take(4 * vn);
    w.dv1 = (uint32_t*)take(4 * vn);
    w.offs = (uint32_t*)take(4 * vn);
    w.tk = (uint32_t*)take(4 * cap);
    w.tv = (uint32_t*)take(4 * cap);
    w.hist = (uint32_t*)take(4ull * (1u << RS_MAX_BITS) * RS_MAX_BLOCKS);
    w.dtot = (uint32_t*)take(4 * (1u << RS_MAX_BITS));
    w.part = (unsigned long long*)take(8 * RS_MAX_BLOCKS);
    w.srect = (int2*)take(8 * vn);
    w.cnt = (uint32_t*)take(4 * 16);
    w.bsrc = (uint32_t*)take(4 * ((size_t)bsrc_last(cap) + 1));
    w.bytes = o;
    return w;
}

int bits_for(unsigned long long n)
{
    int b = 1;
    while (b < 32 && (1ull << b) < n) b++;
    return b;
}

}  // namespace

size_t bin_sort_workspace_size(unsigned long long vn, unsigned long long cap)
{
    return bin_layout(nullptr, vn, cap).bytes;
}

hipError_t launch_bin_sort(const int2* rects, const float* depths, long long N, const ViewTable& vt,
                           unsigned long long cap, void* workspace, uint32_t* isect_tile,
                           uint32_t* isect_gid, int2* ranges, int* info, hipStream_t st)
{
    const unsigned long long vn = (unsigned long long)N * vt.n_views;
    BinWs w = bin_layout((char*)workspace, vn, cap);
    hipError_t e;
    // 1. depth passes over visible (view, Gaussian) pairs
    const int nb_d = sort_blocks(vn);
    SortIO io{};
    io.depths = depths;
    io.rects = rects;
    io.keys_out = w.dk0;
    io.vals_out = w.dv0;
    io.n_const = (uint32_t)vn;
    int dw[4];
    const int dpasses = plan_passes(32, dw);
    if ((e = radix_pass<SRC_PROJ>(io, nb_d, 0, dw[0], w.hist, w.dtot, w.cnt + 0, st)) != hipSuccess) return e;
    uint32_t *ki = w.dk0, *vi = w.dv0, *ko = w.dk1, *vo = w.dv1;
    for (int pass = 1, shift = dw[0]; pass < dpasses; shift += dw[pass], pass++) {
        SortIO p{};
        p.keys_in = ki; p.vals_in = vi; p.vals_out = vo;
        p.keys_out = pass + 1 < dpasses ? ko : nullptr;   // only the order of the last pass is used
        p.n_dev = w.cnt + 0;
        if (pass + 1 == dpasses) {   // the last pass also lays out the rectangles in depth order
            p.rects = rects;
            p.rects_out = w.srect;
        }
        if ((e = radix_pass<SRC_PAIRS>(p, nb_d, shift, dw[pass], w.hist, w.dtot, nullptr, st)) != hipSuccess)
            return e;
        uint32_t* tk = ki; ki = ko; ko = tk;
        uint32_t* tv = vi; vi = vo; vo = tv;
    }
    const uint32_t* pids = vi;   // visible pairs in (depth, view, Gaussian) order

    // 2. scan of tiles_touched in that order
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb_d), dim3(SC_THREADS), 0, st, w.cnt + 0, w.srect, w.part, ranges,
                       (long long)vt.total_tiles);
    hipLaunchKernelGGL(k_scan_down, dim3(nb_d), dim3(SC_THREADS), 0, st, w.srect, w.part, (uint32_t)cap, w.cnt,
                       info, w.offs, w.bsrc, bsrc_last(cap));

    // 3. emission; 4. tile passes (the last one lands in the caller's arrays)
    const int tbits = bits_for((unsigned long long)vt.total_tiles);
    int tw[4];
    const int tpasses = plan_passes(tbits, tw);
    uint32_t *ek = (tpasses % 2 == 0) ? isect_tile : w.tk;
    uint32_t *ev = (tpasses % 2 == 0) ? isect_gid : w.tv;
    const unsigned emit_blocks = (unsigned)((cap + EMIT_SPAN - 1) / EMIT_SPAN);
    // the emission counts the first tile digit when its workgroups fit the
    // histogram's block columns
    const bool fused = emit_blocks <= (unsigned)RS_MAX_BLOCKS;
    hipLaunchKernelGGL(k_emit, dim3(emit_blocks), dim3(EMIT_THREADS), 0, st, pids, w.offs, w.bsrc,
                       bsrc_last(cap), w.cnt, w.srect, N, vt, ek, ev, tw[0], fused ? w.hist : nullptr);
    const int nb_t = sort_blocks(cap);
    uint32_t *tki = ek, *tvi = ev;
    uint32_t *tko = (ek == isect_tile) ? w.tk : isect_tile, *tvo = (ev == isect_gid) ? w.tv : isect_gid;
    for (int pass = 0, shift = 0; pass < tpasses; shift += tw[pass], pass++) {
        SortIO p{};
        p.keys_in = tki; p.vals_in = tvi; p.keys_out = tko; p.vals_out = tvo;
        p.n_dev = w.cnt + 1;
        // a fused first pass takes the emission's histogram, one block per emission workgroup
        const bool pre = fused && pass == 0;
        const int nb = pre ? (int)emit_blocks : nb_t;
        if ((e = radix_pass<SRC_PAIRS>(p, nb, shift, tw[pass], w.hist, w.dtot, nullptr, st, pre)) != hipSuccess)
            return e;
        uint32_t* tk = tki; tki = tko; tko = tk;
        uint32_t* tv = tvi; tvi = tvo; tvo = tv;
    }

    // 5. ranges (zeroed by the scan's first kernel)
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)((cap + 1023) / 1024)), dim3(256), 0, st, isect_tile, w.cnt,
                       (uint32_t)vt.total_tiles, ranges);
    return hipGetLastError();
}

size_t tile_schedule_size(long long total_tiles)
{
    const size_t t = (size_t)total_tiles;
    return align256(4 * t) + align256(4ull * 256 * RS_MAX_BLOCKS) + align256(4 * 256);
}

hipError_t launch_tile_schedule(const int2* ranges, long long total_tiles, void* schedule, hipStream_t st)
{
    char* base = (char*)schedule;
    const size_t t = (size_t)total_tiles;
    uint32_t* order = (uint32_t*)base;
    uint32_t* hist = (uint32_t*)(base + align256(4 * t));
    uint32_t* dtot = (uint32_t*)(base + align256(4 * t) + align256(4ull * 256 * RS_MAX_BLOCKS));
    // one 2048-key chunk per block (a short, latency-bound pass)
    const int nb = (int)min((unsigned long long)RS_MAX_BLOCKS, max(1ull, (t + RS_CHUNK - 1) / RS_CHUNK));
    // one stable 8-bit pass; only the tile ids (the values) are kept
    SortIO a{};
    a.ranges = ranges;
    a.keys_out = nullptr;
    a.vals_out = order;
    a.n_const = (uint32_t)t;
    return radix_pass<SRC_TILE_LEN>(a, nb, 0, 8, hist, dtot, nullptr, st);
}

// order[b] for workgroup b of a grid launch: workgroups are handed to the
// n_xcd XCDs round-robin (b mod n_xcd), so XCD x runs workgroups x, x + n_xcd,
// ...; giving them consecutive tiles keeps neighbouring tiles, which share
// most of their splats, in one XCD's L2
__global__ void k_tile_order_xcd(uint32_t t, int n_xcd, int* __restrict__ order)
{
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= t) return;
    const uint32_t x = b % (uint32_t)n_xcd, q = t / (uint32_t)n_xcd, rem = t % (uint32_t)n_xcd;
    order[b] = (int)(x * q + min(x, rem) + b / (uint32_t)n_xcd);
}

hipError_t launch_tile_order_xcd(long long total_tiles, int n_xcd, void* schedule, hipStream_t st)
{
    const uint32_t t = (uint32_t)total_tiles;
    hipLaunchKernelGGL(k_tile_order_xcd, dim3((t + 255) / 256), dim3(256), 0, st, t, n_xcd, (int*)schedule);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int* p, int value, long long n, hipStream_t st)
{
    return fill_i32(p, value, n, st);
}

size_t morton_workspace_size(long long n)
{
    const size_t t = (size_t)n;
    return 3 * align256(4 * t) + align256(4ull * 256 * RS_MAX_BLOCKS) + align256(4 * 256);
}

// order[i] = index of the Gaussian with the i-th smallest Morton code (stable)
hipError_t launch_morton_order(const float* means, long long n, const float* org, const float* inv_cell,
                               void* workspace, int* order, hipStream_t st)
{
    char* base = (char*)workspace;
    const size_t t = (size_t)n;
    uint32_t* ka = (uint32_t*)base;
    uint32_t* kb = (uint32_t*)(base + align256(4 * t));
    uint32_t* va = (uint32_t*)(base + 2 * align256(4 * t));
    uint32_t* hist = (uint32_t*)(base + 3 * align256(4 * t));
    uint32_t* dtot = (uint32_t*)(base + 3 * align256(4 * t) + align256(4ull * 256 * RS_MAX_BLOCKS));
    const int nb = sort_blocks(t);
    // pass 0 computes the codes from the means; passes 1..3 sort the rest of
    // the 30 bits; the last pass writes the indices into `order`
    SortIO a{};
    a.means = means;
    for (int k = 0; k < 3; k++) { a.org[k] = org[k]; a.inv_cell[k] = inv_cell[k]; }
    a.keys_out = ka;
    a.vals_out = va;
    a.n_const = (uint32_t)t;
    hipError_t e;
    if ((e = radix_pass<SRC_MORTON>(a, nb, 0, 8, hist, dtot, nullptr, st)) != hipSuccess) return e;
    uint32_t *ki = ka, *vi = va, *ko = kb, *vo = (uint32_t*)order;
    for (int pass = 1; pass < 4; pass++) {
        SortIO p{};
        p.keys_in = ki; p.vals_in = vi; p.keys_out = ko; p.vals_out = vo;
        p.n_const = (uint32_t)t;
        if ((e = radix_pass<SRC_PAIRS>(p, nb, 8 * pass, pass == 3 ? 6 : 8, hist, dtot, nullptr, st)) != hipSuccess)
            return e;
        uint32_t* tk = ki; ki = ko; ko = tk;
        uint32_t* tv = vi; vi = vo; vo = tv;
    }
    // after passes 1 (a->b, vals va->order), 2 (b->a, order->va), 3 (a->b, va->order)
    return hipSuccess;
}

namespace {
__global__ void k_gather_columns(const float* __restrict__ src, int C, long long n, const int* __restrict__ order,
                                 float* __restrict__ dst)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long j = order[i];
    // eight planes' loads in flight before their stores
    for (int c0 = 0; c0 < C; c0 += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) v[u] = c0 + u < C ? src[(c0 + u) * n + j] : 0.0f;
#pragma unroll
        for (int u = 0; u < 8; u++)
            if (c0 + u < C) dst[(c0 + u) * n + i] = v[u];
    }
}
}  // namespace

hipError_t launch_gather_columns(const float* src, int C, long long n, const int* order, float* dst, hipStream_t st)
{
    if (n == 0 || C == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_columns, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, C, n, order, dst);
    return hipGetLastError();
}

}  // namespace gs
