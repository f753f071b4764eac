// Cell-linked list on the GPU: hash -> stable radix sort -> reorder + view.
//
// The neighbour set of the method is every j with |r_j - r_i| < 2h
// (Wendland support, Section 2.2).  Particles are binned into cells of edge
// cs >= 2h, so every neighbour lies in the 27 cells around a particle's own.
// Cells are numbered x-fastest, which makes the three cells of a stencil row
// contiguous in sorted order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "common.h"

namespace wcsph {

// ---------------------------------------------------------------- encode

// Key of particle i's cell in its half-row (fluid or boundary) of its
// instance's grid: sorted, each cell row holds its fluid particles, x-cell
// by x-cell, then its boundary particles.  Written by the previous step's
// update where it ran as its own kernel; otherwise computed by the first
// histogram pass of the sort, which stores the keys.
struct EncodeArgs {
    const double *x, *y, *z;
    const uint32_t *id;
    Insts I;
    uint32_t *keys;
};

__device__ __forceinline__ uint32_t encode_key(const EncodeArgs &e, const Inst &ip, int64_t i,
                                               uint32_t id) {
    return sort_key(ip, e.x[i], e.y[i], e.z[i], id);
}

// The keys of a thread's kItems particles (block-strided, 0 past n).  The
// particles of an instance are contiguous in every order the library keeps,
// so a wave's particles nearly always share one instance: it is looked up
// once (from the wave's first particle) and read once for the wave; a wave
// that straddles instances looks them up particle by particle.
template <int kItems>
__device__ __forceinline__ void encode_keys(const EncodeArgs &e, int64_t base, int64_t n,
                                            uint32_t key[kItems]) {
    const int tid = threadIdx.x;
    uint32_t id[kItems];
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int64_t idx = base + (int64_t)it * kSortThreads + tid;
        id[it] = idx < n ? e.id[idx] : 0u;
    }
    int k0 = 0;
    bool one = true;
    if (e.I.n > 1) {
        // items are block-strided: item 0 holds the wave's first particle
        const uint64_t act = __ballot(base + tid < n);
        if (act == 0ull) {  // the wave lies past n: no particle at all
#pragma unroll
            for (int it = 0; it < kItems; ++it) key[it] = 0u;
            return;
        }
        const int l0 = __builtin_amdgcn_readfirstlane(__ffsll((long long)act) - 1);
        k0 = e.I.of_id((uint32_t)__builtin_amdgcn_readlane((int)id[0], l0) & 0x7fffffffu);
        const uint32_t lo = e.I.tab[k0].pstart, hi = e.I.tab[k0].pend;
        bool mine = true;
#pragma unroll
        for (int it = 0; it < kItems; ++it) {
            const uint32_t v = id[it] & 0x7fffffffu;
            mine = mine && (base + (int64_t)it * kSortThreads + tid >= n || (v >= lo && v < hi));
        }
        one = __all(mine);
    }
    if (one) {
        const Inst ip = e.I.get(k0);
#pragma unroll
        for (int it = 0; it < kItems; ++it) {
            const int64_t idx = base + (int64_t)it * kSortThreads + tid;
            key[it] = idx < n ? encode_key(e, ip, idx, id[it]) : 0u;
        }
    } else {
#pragma unroll
        for (int it = 0; it < kItems; ++it) {
            const int64_t idx = base + (int64_t)it * kSortThreads + tid;
            key[it] = idx < n ? encode_key(e, e.I.get(e.I.of_id(id[it] & 0x7fffffffu)), idx, id[it])
                              : 0u;
        }
    }
}

// ------------------------------------------------------ walls in place

// The update flags moving boundary particles (DevScalars::walls_move), which
// only the Verlet update does; the symplectic scheme always gathers every
// particle.
bool walls_in_place_enabled(const Problem &P) {
    return P.scheme == SPH_SCHEME_VERLET && !full_gather();
}

// ------------------------------------------------------------ radix sort
//
// LSD radix sort of (32-bit key, 32-bit index) pairs, 8-bit digits.  Per
// pass: tile histograms -> an exclusive scan of each digit's counts over the
// tiles -> stable scatter (which adds the smaller digits' totals).  Ranks
// inside a tile come from wave-wide digit matching (eight ballots), so a
// tile's keys keep their input order: the sort is stable and deterministic.

// kEncode: the first pass, which computes the keys (encode_key) and stores
// them instead of reading them.
template <int kItems, bool kEncode>
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(const uint32_t *__restrict__ keys,
                                                            int64_t n, int shift,
                                                            uint32_t *__restrict__ hist,
                                                            int ntiles, EncodeArgs e) {
    __shared__ uint32_t h[kRadix];
    const int tid = threadIdx.x;
    for (int d = tid; d < kRadix; d += kSortThreads) h[d] = 0;
    __syncthreads();
    const int tile = tile_of_block(blockIdx.x, ntiles);
    const int64_t base = (int64_t)tile * kSortThreads * kItems;
    uint32_t key[kItems];
    if constexpr (kEncode) {
        encode_keys<kItems>(e, base, n, key);
#pragma unroll
        for (int it = 0; it < kItems; ++it) {
            const int64_t idx = base + (int64_t)it * kSortThreads + tid;
            if (idx < n) e.keys[idx] = key[it];
        }
    } else {
#pragma unroll
        for (int it = 0; it < kItems; ++it) {  // all loads first
            const int64_t idx = base + (int64_t)it * kSortThreads + tid;
            key[it] = idx < n ? keys[idx] : 0u;
        }
    }
#pragma unroll
    for (int it = 0; it < kItems; ++it)
        tile_hist_add(h, key[it], base + (int64_t)it * kSortThreads + tid < n, shift);
    __syncthreads();
    for (int d = tid; d < kRadix; d += kSortThreads) hist[(int64_t)d * ntiles + tile] = h[d];
}

// Exclusive scans (per digit over the tiles for the sort, the chunks per
// half-row).  A block of 1024 threads scans a span of kScanSpan values (4
// consecutive values per thread, wave prefix sums by shuffles, one LDS
// exchange of the 16 wave totals).  launch_scan: up to kScanRedundantSpans
// spans, one launch, block b sums the input before its span itself; up to
// kScanSumSpans, span totals, then block b sums the totals before it and
// scans its span; beyond, span totals -> scan of the totals (one block) ->
// spans scanned with their offsets, all spans in parallel.

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = __lane_id();
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t o = __shfl_up(v, off, kWave);
        if (lane >= off) v += o;
    }
    return v;
}

// Exclusive prefix of v over the block (1024 threads); total = block sum.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *wsum, uint32_t &total) {
    const int t = threadIdx.x, lane = t % kWave, w = t / kWave;
    const uint32_t inc = wave_incl_scan(v);
    if (lane == kWave - 1) wsum[w] = inc;
    __syncthreads();
    if (w == 0) {
        const uint32_t x = lane < kScanThreads / kWave ? wsum[lane] : 0u;
        const uint32_t xi = wave_incl_scan(x);
        if (lane < kScanThreads / kWave) wsum[lane] = xi - x;  // exclusive wave offsets
        if (lane == kScanThreads / kWave - 1) wsum[kScanThreads / kWave] = xi;
    }
    __syncthreads();
    const uint32_t r = wsum[w] + inc - v;
    total = wsum[kScanThreads / kWave];
    __syncthreads();  // wsum may be reused by the next call
    return r;
}

// Loads this thread's 4 values of span `base` (zeros past m).
__device__ __forceinline__ void span_load(const uint32_t *a, int64_t m, int64_t base, uint32_t v[4]) {
    const int64_t i0 = base + 4 * (int64_t)threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = i0 + q < m ? a[i0 + q] : 0u;
}

// Scans span `base` of `in` into `out` (may be the same array) from a
// starting offset; returns the span total.
__device__ __forceinline__ uint32_t span_scan(const uint32_t *in, uint32_t *out, int64_t m,
                                              int64_t base, uint32_t carry, uint32_t *wsum) {
    uint32_t v[4];
    span_load(in, m, base, v);
    const uint32_t tsum = (v[0] + v[1]) + (v[2] + v[3]);
    uint32_t total;
    uint32_t run = carry + block_excl_scan(tsum, wsum, total);
    const int64_t i0 = base + 4 * (int64_t)threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (i0 + q < m) out[i0 + q] = run;
        run += v[q];
    }
    return total;
}

// One block: all spans in order, in place.
__global__ __launch_bounds__(kScanThreads) void k_scan_serial(uint32_t *__restrict__ a, int64_t m) {
    __shared__ uint32_t wsum[kScanThreads / kWave + 1];
    uint32_t carry = 0;
    for (int64_t base = 0; base < m; base += kScanSpan) carry += span_scan(a, a, m, base, carry, wsum);
}

// Block b: the input of spans 0..b-1 summed, then span b scanned from there.
__global__ __launch_bounds__(kScanThreads) void k_scan_redundant(const uint32_t *__restrict__ in,
                                                                 uint32_t *__restrict__ out,
                                                                 int64_t m) {
    __shared__ uint32_t wsum[kScanThreads / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanSpan;  // a multiple of 4096
    const uint4 *in4 = reinterpret_cast<const uint4 *>(in);    // (256-byte aligned arrays)
    const int64_t n4 = base / 4;
    uint32_t p0 = 0, p1 = 0, p2 = 0, p3 = 0;
    int64_t i = threadIdx.x;
    for (; i + 3 * kScanThreads < n4; i += 4 * kScanThreads) {  // four loads in flight
        const uint4 a = in4[i], b = in4[i + kScanThreads];
        const uint4 c = in4[i + 2 * kScanThreads], d = in4[i + 3 * kScanThreads];
        p0 += (a.x + a.y) + (a.z + a.w);
        p1 += (b.x + b.y) + (b.z + b.w);
        p2 += (c.x + c.y) + (c.z + c.w);
        p3 += (d.x + d.y) + (d.z + d.w);
    }
    for (; i < n4; i += kScanThreads) {
        const uint4 a = in4[i];
        p0 += (a.x + a.y) + (a.z + a.w);
    }
    const uint32_t part = (p0 + p1) + (p2 + p3);
    uint32_t offset;
    block_excl_scan(part, wsum, offset);
    span_scan(in, out, m, base, offset, wsum);
}

// Block b: the total of span b.
__global__ __launch_bounds__(kScanThreads) void k_scan_totals(const uint32_t *__restrict__ a,
                                                              int64_t m, uint32_t *__restrict__ tot) {
    __shared__ uint32_t wsum[kScanThreads / kWave + 1];
    uint32_t v[4];
    span_load(a, m, (int64_t)blockIdx.x * kScanSpan, v);
    uint32_t total;
    block_excl_scan((v[0] + v[1]) + (v[2] + v[3]), wsum, total);
    if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

// Block b: span b scanned from its offset (the scanned totals).
__global__ __launch_bounds__(kScanThreads) void k_scan_spans(const uint32_t *__restrict__ in,
                                                             uint32_t *__restrict__ out, int64_t m,
                                                             const uint32_t *__restrict__ off) {
    __shared__ uint32_t wsum[kScanThreads / kWave + 1];
    span_scan(in, out, m, (int64_t)blockIdx.x * kScanSpan, off[blockIdx.x], wsum);
}

// Block b: the totals of spans 0..b-1 summed (a few per thread), then span b
// scanned from there.
__global__ __launch_bounds__(kScanThreads) void k_scan_spans_sum(const uint32_t *__restrict__ in,
                                                                 uint32_t *__restrict__ out,
                                                                 int64_t m,
                                                                 const uint32_t *__restrict__ tot) {
    __shared__ uint32_t wsum[kScanThreads / kWave + 1];
    uint32_t part = 0;
    for (int64_t s = threadIdx.x; s < (int64_t)blockIdx.x; s += kScanThreads) part += tot[s];
    uint32_t offset;
    block_excl_scan(part, wsum, offset);
    span_scan(in, out, m, (int64_t)blockIdx.x * kScanSpan, offset, wsum);
}

// The sort's (digit, tile) counts, digit-major: block d scans digit d's row
// of ntiles counts (its tiles in order, a span at a time) and writes the
// row's total.  The scatter adds the totals of the digits below its own, so
// one launch serves any number of tiles.
__global__ __launch_bounds__(kScanThreads) void k_scan_rows(const uint32_t *__restrict__ in,
                                                            uint32_t *__restrict__ out,
                                                            int64_t ntiles,
                                                            uint32_t *__restrict__ tot) {
    __shared__ uint32_t wsum[kScanThreads / kWave + 1];
    const int64_t row = (int64_t)blockIdx.x * ntiles;
    uint32_t carry = 0;
    for (int64_t base = 0; base < ntiles; base += kScanSpan)
        carry += span_scan(in + row, out + row, ntiles, base, carry, wsum);
    if (threadIdx.x == 0) tot[blockIdx.x] = carry;
}

int launch_scan(const uint32_t *in, uint32_t *out, int64_t m, uint32_t *tot, hipStream_t st) {
    const int64_t spans = (m + kScanSpan - 1) / kScanSpan;
    if (spans <= kScanRedundantSpans) {
        hipLaunchKernelGGL(k_scan_redundant, dim3((unsigned)spans), dim3(kScanThreads), 0, st, in,
                           out, m);
    } else if (spans <= kScanSumSpans) {
        hipLaunchKernelGGL(k_scan_totals, dim3((unsigned)spans), dim3(kScanThreads), 0, st, in, m,
                           tot);
        hipLaunchKernelGGL(k_scan_spans_sum, dim3((unsigned)spans), dim3(kScanThreads), 0, st, in,
                           out, m, tot);
    } else {
        hipLaunchKernelGGL(k_scan_totals, dim3((unsigned)spans), dim3(kScanThreads), 0, st, in, m,
                           tot);
        hipLaunchKernelGGL(k_scan_serial, dim3(1), dim3(kScanThreads), 0, st, tot, spans);
        hipLaunchKernelGGL(k_scan_spans, dim3((unsigned)spans), dim3(kScanThreads), 0, st, in, out,
                           m, tot);
    }
    return launch_check("scan");
}

// Stable scatter of one tile.  Wave w of the tile owns its keys
// [w 64 kItems, (w + 1) 64 kItems) (input order = wave, item, lane), loads
// them all up front, and ranks them item by item against a per-wave digit
// count in LDS that only this wave touches (no workgroup barrier per item).
// One barrier later the per-wave counts become start slots (per digit: the
// keys of all smaller digits, plus its keys in the tiles before this one from
// the row scan, then the waves in order), and every key goes to its slot +
// rank.
template <int kItems>
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout,
    uint32_t *__restrict__ vout, int64_t n, int shift, const uint32_t *__restrict__ hist,
    const uint32_t *__restrict__ dtot, int ntiles) {
    constexpr int kWaves = kSortThreads / kWave;
    static_assert(kSortThreads == kRadix, "one thread per digit for the start slots");
    __shared__ uint32_t wcnt[kWaves][kRadix];  // per-wave counts, then start slots
    __shared__ uint32_t wtot[kWaves];           // digit totals summed per wave
    const int tid = threadIdx.x;
    const int w = tid / kWave, lane = tid % kWave;
    for (int d = lane; d < kRadix; d += kWave) wcnt[w][d] = 0u;
    const int tile = tile_of_block(blockIdx.x, ntiles);
    const int64_t wbase = (int64_t)tile * kSortThreads * kItems + (int64_t)w * kWave * kItems;
    uint32_t key[kItems], val[kItems], rank[kItems];
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int64_t idx = wbase + (int64_t)it * kWave + lane;
        const bool ok = idx < n;
        key[it] = ok ? kin[idx] : 0u;
        val[it] = ok ? (vin ? vin[idx] : (uint32_t)idx) : 0u;
    }
    wave_sync();  // the zeroed counts
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const bool ok = wbase + (int64_t)it * kWave + lane < n;
        const uint32_t d = (key[it] >> shift) & (kRadix - 1);
        // r: earlier lanes of this wave with the same digit; cnt (on the
        // first of them): all of them.  Where the wave's digits do not
        // decrease from lane to lane (nearly sorted keys, the usual case)
        // equal digits are one run of consecutive lanes; else match digits.
        const uint32_t dk = ok ? d : (uint32_t)kRadix;  // kRadix: no key
        uint32_t r, cnt;
        // (the shuffle outside the condition: every lane takes part in it)
        const uint32_t dprev = __shfl_up(dk, 1, kWave);
        if (__ballot(lane > 0 && dk < dprev) == 0) {
            const uint64_t starts = run_starts(dk);
            const uint64_t at_or_below = starts & (lt | (1ull << lane));
            r = (uint32_t)(lane - (63 - __builtin_clzll(at_or_below)));
            cnt = run_length(starts);
        } else {
            const uint64_t peers = match_digit(d, __ballot(ok));
            r = (uint32_t)__popcll(peers & lt);
            cnt = (uint32_t)__popcll(peers);
        }
        const uint32_t before = wcnt[w][d];
        rank[it] = before + r;
        wave_sync();  // every lane has read before the leader updates
        if (ok && r == 0) wcnt[w][d] = before + cnt;
        wave_sync();
    }
    // the keys of all smaller digits come first: an exclusive scan of the
    // digit totals over the block (by waves, then the wave totals; loaded
    // here, as a load issued before the keys' would delay their wait)
    const uint32_t dt = dtot[tid];
    const uint32_t dincl = wave_incl_scan(dt);
    if (lane == kWave - 1) wtot[w] = dincl;
    __syncthreads();
    {
        const int d = tid;
        uint32_t run = hist[(int64_t)d * ntiles + tile] + (dincl - dt);
#pragma unroll
        for (int k = 0; k < kWaves - 1; ++k) run += k < w ? wtot[k] : 0u;
#pragma unroll
        for (int k = 0; k < kWaves; ++k) {
            const uint32_t c = wcnt[k][d];
            wcnt[k][d] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const bool ok = wbase + (int64_t)it * kWave + lane < n;
        if (ok) {
            const uint32_t d = (key[it] >> shift) & (kRadix - 1);
            const uint32_t pos = wcnt[w][d] + rank[it];
            kout[pos] = key[it];
            vout[pos] = val[it];
        }
    }
}

// full: sort on every key bit; else on the cell key only (the sub-cell bits
// keep the order of the input).  keys (KeysLeft): kKeysOnly, w.keys_next()
// holds the keys of the current positions; kKeysCounted, w.hist() also holds
// the first pass's digit counts (both for this step's `full`); kNoKeys, the
// first histogram pass computes the keys and counts them.
int launch_sort(const Problem &P, const sph_state &s, const Ws &w, hipStream_t st, bool full,
                int keys, uint32_t **sorted_keys, uint32_t **perm) {
    const int64_t n = w.L.n;
    const int ntiles = (int)w.L.ntiles;
    const int low = full ? 0 : kSubBits;
    const int bits = w.L.key_bits - low;
    const int passes = bits <= 0 ? 1 : (bits + kRadixBits - 1) / kRadixBits;
    const bool small = sort_tile(n) == (int64_t)kSortThreads * kSortItemsSmall;
    uint32_t *kin = w.keys_next();
    uint32_t *kout = (passes & 1) ? w.keys() : w.keys_alt();
    uint32_t *kother = (passes & 1) ? w.keys_alt() : w.keys();  // the ping-pong's second buffer
    uint32_t *vbuf[2] = {w.vals(), w.vals_alt()};
    uint32_t *vin = nullptr;  // first pass ranks the identity permutation
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = low + pass * kRadixBits;
        uint32_t *vout = vbuf[pass & 1];
        const EncodeArgs e{s.x, s.y, s.z, s.id, insts_of(P, w), kin};
        const bool encode = pass == 0 && keys == kNoKeys;
        // the update kernel has also counted the first pass's digits
        const bool counted = pass == 0 && keys == kKeysCounted;
        if (!counted && small) {
            if (encode)
                hipLaunchKernelGGL((k_sort_hist<kSortItemsSmall, true>), dim3(ntiles),
                                   dim3(kSortThreads), 0, st, kin, n, shift, w.hist(), ntiles, e);
            else
                hipLaunchKernelGGL((k_sort_hist<kSortItemsSmall, false>), dim3(ntiles),
                                   dim3(kSortThreads), 0, st, kin, n, shift, w.hist(), ntiles, e);
        } else if (!counted) {
            if (encode)
                hipLaunchKernelGGL((k_sort_hist<kSortItemsLarge, true>), dim3(ntiles),
                                   dim3(kSortThreads), 0, st, kin, n, shift, w.hist(), ntiles, e);
            else
                hipLaunchKernelGGL((k_sort_hist<kSortItemsLarge, false>), dim3(ntiles),
                                   dim3(kSortThreads), 0, st, kin, n, shift, w.hist(), ntiles, e);
        }
        hipLaunchKernelGGL(k_scan_rows, dim3(kRadix), dim3(kScanThreads), 0, st, w.hist(),
                           w.hist_off(), (int64_t)ntiles, w.hist_tot());
        if (small)
            hipLaunchKernelGGL(k_sort_scatter<kSortItemsSmall>, dim3(ntiles), dim3(kSortThreads),
                               0, st, kin, vin, kout, vout, n, shift, w.hist_off(), w.hist_tot(),
                               ntiles);
        else
            hipLaunchKernelGGL(k_sort_scatter<kSortItemsLarge>, dim3(ntiles), dim3(kSortThreads),
                               0, st, kin, vin, kout, vout, n, shift, w.hist_off(), w.hist_tot(),
                               ntiles);
        if (int rc = launch_check("radix sort")) return rc;
        kin = kout;
        kout = kother;
        kother = kin;
        vin = vout;
    }
    *sorted_keys = kin;
    *perm = vin;
    return 0;
}

// ------------------------------------------------------------ cell table

// start[k] = first sorted position whose cell key >= k, for k in [0, 2 ncells]
// (lower bound; an empty cell gets the start of the next one).  Cells x0..x1
// of a half-row with key k0 at x = 0 hold the sorted range
// [start[k0 + x0], start[k0 + x1 + 1]).  The search starts from the entry's
// previous value (particles move little between steps, so it is usually
// exact or close): gallop away from it until the answer is bracketed, then
// bisect.  The hint only changes the cost: any value gives the exact bound.
__device__ __forceinline__ void cell_table_entry(const uint32_t *__restrict__ keys, int64_t n, int64_t c,
                                 uint32_t *__restrict__ start) {
    const int64_t h = start[c] < (uint64_t)n ? (int64_t)start[c] : n;
    int64_t lo, hi;  // the answer lies in [lo, hi]
    if (h < n && (int64_t)key_cell(keys[h]) < c) {
        lo = h + 1;
        hi = n;
        for (int64_t step = 1;; step <<= 1) {
            const int64_t q = h + step;
            if (q >= n) break;
            if ((int64_t)key_cell(keys[q]) >= c) {
                hi = q;
                break;
            }
            lo = q + 1;
        }
    } else {
        lo = 0;
        hi = h;
        for (int64_t step = 1;; step <<= 1) {
            const int64_t q = h - step;
            if (q < 0) break;
            if ((int64_t)key_cell(keys[q]) < c) {
                lo = q + 1;
                break;
            }
            hi = q;
        }
    }
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if ((int64_t)key_cell(keys[mid]) < c)
            lo = mid + 1;
        else
            hi = mid;
    }
    start[c] = (uint32_t)lo;
}


// ----------------------------------------------------- reorder and view

struct ReorderArgs {
    const uint32_t *perm;
    const uint32_t *keys;
    int64_t n;
    // source arrays
    const double *x, *y, *z, *ux, *uy, *uz, *uxm, *uym, *uzm;
    const void *rho, *rhom;
    const uint32_t *id;
    // destination arrays
    double *x2, *y2, *z2, *ux2, *uy2, *uz2, *uxm2, *uym2, *uzm2;
    void *rho2, *rhom2;
    uint32_t *id2;
    // view
    void *v0, *v1, *v2;
    Insts I;
    // cell table, built by the first table_blocks blocks
    uint32_t *start;
    int64_t nkeys;
    uint32_t table_blocks;
    WallsInPlace wip;  // on: boundary particles stay (the sort left them in place)
};

// Offset of coordinate v from the centre of cell c, computed in FP64 with
// one rounding per operation (no contraction) and rounded once to FP32.
__device__ __forceinline__ float cell_offset(double v, double o, int c, double cs) {
#pragma clang fp contract(off)
    double t = v - o;
    double ctr = ((double)c + 0.5) * cs;
    return (float)(t - ctr);
}

// Tait pressure and sound speed of the mixed view from rho - rho0 (FP32).
template <bool kGamma7>
__device__ __forceinline__ void mixed_eos(const Inst &ip, float dr, double &P, double &cs) {
    const double xr = (double)dr / ip.rho0;
    if constexpr (kGamma7) {
        const double q = xr * (7.0 + xr * (21.0 + xr * (35.0 + xr * (35.0 + xr * (21.0 + xr * (7.0 + xr))))));
        P = ip.B * q;
        cs = ip.c_const ? ip.c0 : ip.c0 * (1.0 + xr * (3.0 + xr * (3.0 + xr)));
    } else {
        const double l1p = log1p(xr);
        P = ip.B * expm1(ip.gamma * l1p);
        cs = ip.c_const ? ip.c0 : ip.c0 * exp(0.5 * (ip.gamma - 1.0) * l1p);
    }
}

// Gathers the state into cell order and writes the interaction view:
// mixed: {offset from the cell centre (FP32), u_x}, {u_y, u_z}, {rho - rho0,
// P, 1/rho, +-c} (what a fixed wall changes from step to step is in the last
// vector alone); FP64: {r, rho}, {u, P}, {1/rho, +-c}; c < 0 marks a boundary
// particle.  P from the Tait equation, c the Tait sound speed (or c0).
// Mixed precision takes them from x = (rho - rho0) / rho0 in FP64 without
// cancellation: (1 + x)^gamma - 1 = expm1(gamma log1p(x)); kGamma7 (every
// instance has gamma = 7, the value of all the paper's runs) expands the
// binomial instead, x (7 + 21 x + ... + x^6) and c0 (1 + x)^3, which needs no
// transcendental calls and fewer registers.
// The same launch also builds the cell table from the sorted keys (the two
// are independent): its first table_blocks blocks compute the entries (they
// are latency-bound searches, dispatched first so that they overlap the
// gather).
// With fixed walls in place a boundary particle keeps its sorted position: both
// buffers of x, u, um and id already hold its values there (the two steps
// before gathered every particle, and a fixed wall's position and zero
// velocity never change), so only the densities (which the update changed)
// are copied and the view's density-dependent part rewritten (mixed: the
// offsets and zero velocity stay from the step before, at the same position;
// FP64: the whole view, u = 0).  reorder_one: position k, with its key's
// cell and its instance.
template <bool kMixed, bool kGamma7>
__device__ __forceinline__ void reorder_one(const ReorderArgs &a, int64_t k, uint32_t key,
                                            const Inst &ip) {
    uint32_t off = key - 2u * ip.cell_base;  // half cells + lrow nx + cx
    const bool bhalf = off >= inst_cells(ip);
    if (bhalf) off -= inst_cells(ip);
    const uint32_t lrow = off / (uint32_t)ip.nx;
    const int cx = (int)(off % (uint32_t)ip.nx);
    const int cy = (int)(lrow % (uint32_t)ip.ny);
    const int cz = (int)(lrow / (uint32_t)ip.ny);
    if (bhalf && a.wip.on()) {
        if constexpr (kMixed) {
            // the view's offsets and (zero) velocity are those of the step
            // before; the update also wrote both density levels to the
            // destination buffers
            const float dr = static_cast<const float *>(a.rho)[k];
            double P, cs;
            mixed_eos<kGamma7>(ip, dr, P, cs);
            const double inv = 1.0 / (ip.rho0 + (double)dr);
            static_cast<float4 *>(a.v2)[k] = make_float4(dr, (float)P, (float)inv, -(float)cs);
        } else {
            const double x = a.x[k], y = a.y[k], z = a.z[k];
            const double rho = static_cast<const double *>(a.rho)[k];
            static_cast<double *>(a.rho2)[k] = rho;
            static_cast<double *>(a.rhom2)[k] = static_cast<const double *>(a.rhom)[k];
            const double r = rho / ip.rho0;
            const double P = ip.B * (pow(r, ip.gamma) - 1.0);
            const double cs = ip.c_const ? ip.c0 : ip.c0 * pow(r, 0.5 * (ip.gamma - 1.0));
            static_cast<double4 *>(a.v0)[k] = make_double4(x, y, z, rho);
            static_cast<double4 *>(a.v1)[k] = make_double4(0.0, 0.0, 0.0, P);
            static_cast<double2 *>(a.v2)[k] = make_double2(1.0 / rho, -cs);
        }
        return;
    }
    const uint32_t src = a.perm[k];
    const double x = a.x[src], y = a.y[src], z = a.z[src];
    const double ux = a.ux[src], uy = a.uy[src], uz = a.uz[src];
    const uint32_t id = a.id[src];
    a.x2[k] = x;
    a.y2[k] = y;
    a.z2[k] = z;
    a.ux2[k] = ux;
    a.uy2[k] = uy;
    a.uz2[k] = uz;
    a.uxm2[k] = a.uxm[src];
    a.uym2[k] = a.uym[src];
    a.uzm2[k] = a.uzm[src];
    a.id2[k] = id;
    const bool bnd = (id >> 31) != 0;
    if constexpr (kMixed) {
        const float dr = static_cast<const float *>(a.rho)[src];
        static_cast<float *>(a.rho2)[k] = dr;
        static_cast<float *>(a.rhom2)[k] = static_cast<const float *>(a.rhom)[src];
        double P, cs;
        mixed_eos<kGamma7>(ip, dr, P, cs);
        const double inv = 1.0 / (ip.rho0 + (double)dr);
        static_cast<float4 *>(a.v0)[k] =
            make_float4(cell_offset(x, ip.ox, cx, ip.cs), cell_offset(y, ip.oy, cy, ip.cs),
                        cell_offset(z, ip.oz, cz, ip.cs), (float)ux);
        static_cast<float2 *>(a.v1)[k] = make_float2((float)uy, (float)uz);
        static_cast<float4 *>(a.v2)[k] =
            make_float4(dr, (float)P, (float)inv, bnd ? -(float)cs : (float)cs);
    } else {
        const double rho = static_cast<const double *>(a.rho)[src];
        static_cast<double *>(a.rho2)[k] = rho;
        static_cast<double *>(a.rhom2)[k] = static_cast<const double *>(a.rhom)[src];
        const double r = rho / ip.rho0;
        const double P = ip.B * (pow(r, ip.gamma) - 1.0);
        const double cs = ip.c_const ? ip.c0 : ip.c0 * pow(r, 0.5 * (ip.gamma - 1.0));
        double4 v0 = make_double4(x, y, z, rho);
        double4 v1 = make_double4(ux, uy, uz, P);
        double2 v2 = make_double2(1.0 / rho, bnd ? -cs : cs);
        static_cast<double4 *>(a.v0)[k] = v0;
        static_cast<double4 *>(a.v1)[k] = v1;
        static_cast<double2 *>(a.v2)[k] = v2;
    }
}

template <bool kMixed, bool kGamma7>
__global__ void k_reorder(ReorderArgs a) {
    if (blockIdx.x < a.table_blocks) {
        const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (c <= a.nkeys) cell_table_entry(a.keys, a.n, c, a.start);
        return;
    }
    int64_t k = (int64_t)(blockIdx.x - a.table_blocks) * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const uint32_t key = key_cell(a.keys[k]);
    reorder_one<kMixed, kGamma7>(a, k, key, a.I.get(a.I.of_cell(key_row_cell(key))));
}

int launch_reorder(const Problem &P, sph_state &s, const Ws &w, const uint32_t *keys,
                   const uint32_t *perm, bool walls_in_place, hipStream_t st) {
    ReorderArgs a;
    a.perm = perm;
    a.keys = keys;
    a.n = s.n;
    a.x = s.x; a.y = s.y; a.z = s.z;
    a.ux = s.ux; a.uy = s.uy; a.uz = s.uz;
    a.uxm = s.uxm; a.uym = s.uym; a.uzm = s.uzm;
    a.rho = s.rho; a.rhom = s.rhom; a.id = s.id;
    a.x2 = s.x_alt; a.y2 = s.y_alt; a.z2 = s.z_alt;
    a.ux2 = s.ux_alt; a.uy2 = s.uy_alt; a.uz2 = s.uz_alt;
    a.uxm2 = s.uxm_alt; a.uym2 = s.uym_alt; a.uzm2 = s.uzm_alt;
    a.rho2 = s.rho_alt; a.rhom2 = s.rhom_alt; a.id2 = s.id_alt;
    a.v0 = w.base + w.L.view0;
    a.v1 = w.base + w.L.view1;
    a.v2 = w.base + w.L.view2;
    a.I = insts_of(P, w);
    a.start = w.cell_start();
    a.nkeys = 2 * w.L.ncells;
    a.table_blocks = (uint32_t)((a.nkeys + 1 + 255) / 256);
    a.wip.walls = &w.scalars()->walls_move;
    a.wip.allow = walls_in_place && walls_in_place_enabled(P) ? 1 : 0;
    const int blocks = (int)(a.table_blocks + (s.n + 255) / 256);
    bool g7 = true;
    for (const Inst &ip : P.host) g7 = g7 && ip.gamma == 7.0;
    if (P.precision == SPH_MIXED && g7)
        hipLaunchKernelGGL((k_reorder<true, true>), dim3(blocks), dim3(256), 0, st, a);
    else if (P.precision == SPH_MIXED)
        hipLaunchKernelGGL((k_reorder<true, false>), dim3(blocks), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_reorder<false, false>), dim3(blocks), dim3(256), 0, st, a);
    if (int rc = launch_check("reorder")) return rc;
    // the gathered arrays are now current
    auto swp = [](auto &u, auto &v) { auto t = u; u = v; v = t; };
    swp(s.x, s.x_alt); swp(s.y, s.y_alt); swp(s.z, s.z_alt);
    swp(s.ux, s.ux_alt); swp(s.uy, s.uy_alt); swp(s.uz, s.uz_alt);
    swp(s.uxm, s.uxm_alt); swp(s.uym, s.uym_alt); swp(s.uzm, s.uzm_alt);
    swp(s.rho, s.rho_alt); swp(s.rhom, s.rhom_alt); swp(s.id, s.id_alt);
    return 0;
}

// ------------------------------------------------------------ chunk list
//
// The interaction works on chunks: up to csz (64, or the group size of the
// group-per-wave kernels) consecutive sorted particles of one half-row (the
// fluid or the boundary particles of a cell row, fixed cy and cz) of one
// instance, so a chunk is all fluid or all boundary.  Per half-row: the
// number of its chunks (k_row_counts), an exclusive scan of those numbers
// (the first chunk of every half-row), then the chunks {start, end, local
// half-row 2 lrow + half, instance} and the chunk count (k_row_chunks).
//
// k_row_counts also prepares the per-instance time-step bound for the
// interaction that follows: the bound of the last interaction (if there was
// one) becomes the lagged bound, and the running minimum restarts at +inf.
// With `lagged` it also sets this step's dt before the interaction runs:
// the caller's dt, else Cr times the lagged bound (eq. sphdt one step late);
// with no bound yet, dt = 0 and the CFL flag is raised.

// Instance of global row `row`, the same in every lane of the wave (all
// lanes active): the instances' first rows do not decrease, so the answer is
// the number of instances starting at or below `row`, less one; the wave
// reads 64 of them at a time and counts with a ballot (one load latency
// instead of a binary search's chain of dependent loads).
__device__ __forceinline__ int of_row_wave(const Insts &I, uint32_t row) {
    if (I.n == 1) return 0;
    const int lane = threadIdx.x % kWave;
    int below = 0;
    for (int b = 0; b < I.n; b += kWave) {
        const int k = b + lane;
        const int c = __popcll(__ballot(k < I.n && I.tab[k < I.n ? k : 0].row_base <= row));
        below += c;
        if (c < kWave) break;  // (uniform) every later instance starts above `row`
    }
    return below - 1;
}

// Global half-row r (row r / 2, half r % 2; the same in every lane of the
// wave): its instance, local half-row and the key of its cell x = 0.
__device__ __forceinline__ void half_row(const Insts &I, int64_t r, int &inst, int &lhalf,
                                         uint32_t &k0, int &nx) {
    inst = of_row_wave(I, (uint32_t)(r >> 1));
    const Inst ip = I.get(inst);
    lhalf = (int)(r - 2 * (int64_t)ip.row_base);
    k0 = half_row_key(ip, (uint32_t)lhalf >> 1, (uint32_t)lhalf & 1u);
    nx = ip.nx;
}

// The chunks of a half-row (cells k0 .. k0 + nx - 1): its runs of
// consecutive non-empty cells, each cut into pieces of csz particles, so that
// no chunk spans empty cells (a chunk with a gap inside streams every
// candidate across the gap).  A run ends at an empty cell only while the
// half-row keeps within ceil(particles / csz) + 1 chunks; past that budget a
// chunk spans the gap, and the total stays below a fixed bound.  The rule is
// sequential in x (the budget left depends on the runs before), so the 64
// lanes of a wave load 64 cells at a time and one scalar loop visits the
// gaps in order (a run can only end at an empty cell after a non-empty one;
// later cells of the same gap would give the same answer).  Calls
// emit(k, r0, r1) (all lanes, uniform arguments) for every run [r0, r1)
// whose first chunk is chunk k; returns the chunk count.
__device__ __forceinline__ uint32_t pieces(uint32_t len, uint32_t csz) {
    return (len + csz - 1) / csz;
}

template <class F>
__device__ __forceinline__ uint32_t half_row_chunks(const uint32_t *__restrict__ start,
                                                    uint32_t k0, int nx, uint32_t csz, F emit) {
    const int lane = threadIdx.x % kWave;
    const uint32_t b = start[k0], e = start[k0 + nx];
    const uint32_t budget = pieces(e - b, csz) + 1;
    uint32_t used = 0, run0 = b;
    for (int x0 = 0; x0 < nx; x0 += kWave) {
        const int x = x0 + lane;
        bool ev = false;
        uint32_t p0 = 0;
        if (x >= 1 && x < nx) {
            const uint32_t pm = start[k0 + x - 1];
            p0 = start[k0 + x];
            const uint32_t p1 = start[k0 + x + 1];
            ev = p1 == p0 && p0 > pm;  // cell x empty, cell x - 1 not
        }
        uint64_t m = __ballot(ev);
        while (m) {
            const int l = __ffsll((long long)m) - 1;
            m &= m - 1;
            const uint32_t prev = (uint32_t)__shfl((int)p0, l, kWave);
            const uint32_t k = pieces(prev - run0, csz);
            if (prev > run0 && used + k + pieces(e - prev, csz) <= budget) {
                emit(used, run0, prev);
                used += k;
                run0 = prev;
            }
        }
    }
    emit(used, run0, e);
    return used + pieces(e - run0, csz);
}

// One wave per half-row (wave index = half-row); the first threads also
// advance the instances' clocks.
__global__ __launch_bounds__(256) void k_row_counts(const uint32_t *__restrict__ start, Insts I,
                                                    int64_t nhalf, uint32_t csz,
                                                    uint32_t *__restrict__ cnt, DevScalars *sc,
                                                    InstState *ist, int lagged, double dt_arg,
                                                    uint32_t *__restrict__ zero, int64_t nzero) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < nzero) zero[g] = 0u;  // digit counts the fused interaction adds to
    if (g == 0 && lagged) sc->steps += 1;
    constexpr unsigned long long kInf = 0x7ff0000000000000ull;
    if (g < I.n) {
        const int k = (int)g;
        if (ist[k].dt_min_bits != kInf) ist[k].dt_lag_bits = ist[k].dt_min_bits;
        ist[k].dt_min_bits = kInf;
        if (lagged) {
            const double cfl = I.get(k).cfl;
            const unsigned long long lb = ist[k].dt_lag_bits;
            const double bound = cfl * __longlong_as_double((long long)lb);
            double dt = dt_arg > 0.0 ? dt_arg : bound;
            if (lb == kInf) {
                if (!(dt_arg > 0.0)) dt = 0.0;
                sc->dt_cfl_violation = 1u;
            } else if (dt > bound) {
                sc->dt_cfl_violation = 1u;
            }
            ist[k].dt_cfl = bound;
            ist[k].dt_last = dt;
            ist[k].time += dt;
        }
    }
    const int64_t r = g / kWave;
    if (r >= nhalf) return;  // whole waves
    int inst, lhalf, nx;
    uint32_t k0;
    half_row(I, r, inst, lhalf, k0, nx);
    const uint32_t nch = half_row_chunks(start, k0, nx, csz, [](uint32_t, uint32_t, uint32_t) {});
    if (g % kWave == 0) cnt[r] = nch;
}

// kScan: `first` holds the chunk counts themselves (few half-rows): the block
// sums the counts of the half-rows before its own (each thread a strided
// share), and each wave adds those of the block's waves before it.
constexpr int kRowScanMax = 4096;  // half-rows up to which k_row_chunks scans itself
template <bool kScan>
__global__ __launch_bounds__(256) void k_row_chunks(const uint32_t *__restrict__ start, Insts I,
                                                    int64_t nhalf, uint32_t csz,
                                                    const uint32_t *__restrict__ first,
                                                    int4 *__restrict__ chunks, DevScalars *sc) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t r = g / kWave;
    uint32_t f = 0;
    if constexpr (kScan) {
        __shared__ uint32_t part[256 / kWave];
        const int64_t r0 = (int64_t)blockIdx.x * (256 / kWave);  // the block's first half-row
        uint32_t s = 0;
        for (int64_t q = threadIdx.x; q < r0; q += 256) s += first[q];
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) s += __shfl_xor(s, off, kWave);
        const int w = threadIdx.x / kWave;
        if (threadIdx.x % kWave == 0) part[w] = s;
        __syncthreads();
        f = part[0] + part[1] + part[2] + part[3];
        for (int64_t q = r0; q < r && q < nhalf; ++q) f += first[q];
    }
    if (r >= nhalf) return;  // whole waves
    const int lane = (int)(g % kWave);
    int inst, lhalf, nx;
    uint32_t k0;
    half_row(I, r, inst, lhalf, k0, nx);
    if constexpr (!kScan) f = first[r];
    const uint32_t nch =
        half_row_chunks(start, k0, nx, csz, [&](uint32_t k, uint32_t r0, uint32_t r1) {
            const uint32_t np = pieces(r1 - r0, csz);
            for (uint32_t q = (uint32_t)lane; q < np; q += kWave) {
                const uint32_t s0 = r0 + q * csz;
                chunks[f + k + q] = make_int4((int)s0, (int)(s0 + csz < r1 ? s0 + csz : r1), lhalf, inst);
            }
        });
    if (r == nhalf - 1 && lane == 0) sc->nchunks = f + nch;
}

int launch_chunks(const Problem &P, const Ws &w, bool lagged, double dt, hipStream_t st,
                  bool zero_hist) {
    const int64_t nhalf = 2 * w.L.nrows;
    const int64_t nzero = zero_hist ? (int64_t)kRadix * w.L.ntiles : 0;
    const int64_t threads =
        std::max<int64_t>(std::max<int64_t>(nhalf * kWave, (int64_t)P.host.size()), nzero);
    const int blocks = (int)((threads + 255) / 256);
    const Insts I = insts_of(P, w);
    const uint32_t csz = (uint32_t)chunk_for(P);
    hipLaunchKernelGGL(k_row_counts, dim3(blocks), dim3(256), 0, st, w.cell_start(), I, nhalf,
                       csz, w.row_cnt(), w.scalars(), w.inst_state(), (int)lagged, dt, w.hist(),
                       nzero);
    if (int rc = launch_check("chunk counts")) return rc;
    const dim3 grid((unsigned)((nhalf * kWave + 255) / 256));
    if (nhalf <= kRowScanMax) {
        hipLaunchKernelGGL(k_row_chunks<true>, grid, dim3(256), 0, st, w.cell_start(), I, nhalf,
                           csz, w.row_cnt(), w.chunks(), w.scalars());
    } else {
        if (int rc = launch_scan(w.row_cnt(), w.row_first(), nhalf, w.scan_tot(), st)) return rc;
        hipLaunchKernelGGL(k_row_chunks<false>, grid, dim3(256), 0, st, w.cell_start(), I, nhalf,
                           csz, w.row_first(), w.chunks(), w.scalars());
    }
    return launch_check("chunk list");
}

}  // namespace wcsph
