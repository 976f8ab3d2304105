// Binning of visibilities by (w-plane, uv tile, edge region): the MI355X
// counterpart of the paper's per-slab linked lists (Sec. 3.2), which gather
// the visibilities of one slab, halo included, into contiguous arrays so
// that the gridding kernel reads them in order.  Here a counting sort builds
// one contiguous record range per key:
//   bin_count   FP64 placement, key and rank of every visibility; ranks
//               come from an LDS hash table per workgroup, so a hot key
//               costs one global atomic per workgroup, not per visibility
//   scan_*      exclusive scan of the key counts into record offsets
//   bin_scatter writes the packed record of every visibility at
//               offset[key] + rank
//   tile_work   per tile: records to process (own + neighbours' facing
//               strips), number of work items, split-tile scratch slots
#include "ws_kernels.h"

namespace ws {

namespace {

constexpr int kCountThreads = 256;
constexpr int kCountPerBlock = 4096;    // visibilities per workgroup
constexpr int kHashSize = 8192;         // >= 2 x kCountPerBlock
static_assert(kHashSize == 1 << 13, "hash_slot takes 13 bits");
constexpr int kCountPerThread = kCountPerBlock / kCountThreads;

__device__ __forceinline__ uint32_t hash_slot(uint32_t key) {
  return (key * 2654435761u) >> (32 - 13);  // 13 = log2(kHashSize)
}

// Speed of light (m/s): baseline-major uvw in metres becomes wavelengths
// at frequency f by the factor f / c0.
constexpr double kSpeedOfLight = 299792458.0;

// Baseline coordinates of visibility i in wavelengths.  Baseline-major:
// the scale f / c0 is one FP64 division, then one product per coordinate
// (contraction off, so the position rounds as the separate operations).
__device__ __forceinline__ void source_uvw(const VisSource& s, int64_t i,
                                           double& u, double& v, double& w) {
#pragma clang fp contract(off)
  if (s.rows) {
    const int64_t r = i / s.nchan;
    const int c = (int)(i - r * s.nchan);
    const double sc = s.freq[c] / kSpeedOfLight;
    u = s.uvw[3 * r] * sc;
    v = s.uvw[3 * r + 1] * sc;
    w = s.uvw[3 * r + 2] * sc;
  } else {
    u = s.uvw[3 * i];
    v = s.uvw[3 * i + 1];
    w = s.uvw[3 * i + 2];
  }
}

// Weighted value of visibility i (gridding).  Baseline-major: the
// correlations of row r, channel c combined in FP64 with the coefficients
// and the per-correlation weights, then rounded to the path precision.
template <typename R>
__device__ __forceinline__ cplx<R> source_value(const VisSource& s,
                                                int64_t i) {
  if (s.rows) {
    const int64_t r = i / s.nchan;
    const cplx<R>* v = static_cast<const cplx<R>*>(s.vis) + i * s.npol;
    double re = 0.0, im = 0.0;
    for (int p = 0; p < s.npol; ++p) {
      const double wt = s.weight != nullptr
                            ? (double)s.weight[r * s.npol + p] : 1.0;
      const double ar = s.coef[p][0] * wt, ai = s.coef[p][1] * wt;
      const cplx<R> x = v[p];
      re += ar * (double)x.re - ai * (double)x.im;
      im += ar * (double)x.im + ai * (double)x.re;
    }
    return {(R)re, (R)im};
  }
  const R wt = s.weight != nullptr ? (R)s.weight[i] : (R)1;
  if (s.vis == nullptr) return {wt, (R)0};  // unit visibilities
  const cplx<R> vv = static_cast<const cplx<R>*>(s.vis)[i];
  return {wt * vv.re, wt * vv.im};
}

// Weight of visibility i (degridding reads flat sources only).
__device__ __forceinline__ float source_weight(const VisSource& s,
                                               int64_t i) {
  return s.weight != nullptr ? s.weight[i] : 1.0f;
}

__global__ __launch_bounds__(kCountThreads) void k_bin_count(
    Geo g, VisSource src, int64_t m,
    uint32_t* __restrict__ copies, uint32_t nkeys,
    uint2* __restrict__ keyrank, unsigned long long* __restrict__ dropped) {
  uint32_t* __restrict__ counts =
      copies + (size_t)(blockIdx.x % kCountCopies) * nkeys;
  __shared__ uint32_t s_key[kHashSize];
  __shared__ uint32_t s_cnt[kHashSize];
  __shared__ unsigned long long s_drop;
  const int tid = threadIdx.x;
  for (int s = tid; s < kHashSize; s += kCountThreads) {
    s_key[s] = kNoKey;
    s_cnt[s] = 0;
  }
  if (tid == 0) s_drop = 0;
  __syncthreads();

  uint32_t my_key[kCountPerThread];
  uint32_t my_slot[kCountPerThread];
  uint32_t my_rank[kCountPerThread];
  unsigned long long my_drop = 0;
  const int64_t base = (int64_t)blockIdx.x * kCountPerBlock;
  // All coordinates first (indices clamped into range), so that the loads
  // overlap instead of each waiting behind the previous one's LDS atomics.
  double cu[kCountPerThread], cv[kCountPerThread], cw[kCountPerThread];
#pragma unroll
  for (int e = 0; e < kCountPerThread; ++e) {
    int64_t gi = base + e * kCountThreads + tid;
    gi = gi < m ? gi : m - 1;
    source_uvw(src, gi, cu[e], cv[e], cw[e]);
  }
#pragma unroll
  for (int e = 0; e < kCountPerThread; ++e) {
    const int64_t gi = base + e * kCountThreads + tid;
    my_key[e] = kNoKey;
    if (gi < m) {
      double x, y;
      int i0, j0, k;
      const double u = cu[e], v = cv[e], w = cw[e];
      if (place(g, u, v, w, x, y, i0, j0, k)) {
        my_drop += (unsigned long long)(g.K * g.K - taps_on_grid(g, i0, j0));
        const uint32_t key = bin_key(g, i0, j0, k);
        uint32_t s = hash_slot(key);
        while (true) {
          const uint32_t prev = atomicCAS(&s_key[s], kNoKey, key);
          if (prev == kNoKey || prev == key) break;
          s = (s + 1) & (kHashSize - 1);
        }
        my_key[e] = key;
        my_slot[e] = s;
        my_rank[e] = atomicAdd(&s_cnt[s], 1u);
      } else {
        my_drop += (unsigned long long)(g.K * g.K);
      }
    }
  }
  if (dropped != nullptr && my_drop != 0) atomicAdd(&s_drop, my_drop);
  __syncthreads();
  // One global atomic per distinct key of the workgroup; the returned old
  // count becomes the workgroup's base rank for that key (kept in s_cnt).
  // All of a thread's atomics are issued before any result is used, so
  // their round trips overlap.
  constexpr int kSlotsPerThread = kHashSize / kCountThreads;
  uint32_t old[kSlotsPerThread];
#pragma unroll
  for (int e = 0; e < kSlotsPerThread; ++e) {
    const int s = tid + e * kCountThreads;
    const uint32_t key = s_key[s];
    old[e] = key != kNoKey ? atomicAdd(&counts[key], s_cnt[s]) : 0u;
  }
#pragma unroll
  for (int e = 0; e < kSlotsPerThread; ++e) {
    const int s = tid + e * kCountThreads;
    if (s_key[s] != kNoKey) s_cnt[s] = old[e];
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < kCountPerThread; ++e) {
    const int64_t gi = base + e * kCountThreads + tid;
    if (gi < m) {
      uint2 kr;
      kr.x = my_key[e];
      kr.y = my_key[e] == kNoKey ? 0u : s_cnt[my_slot[e]] + my_rank[e];
      keyrank[gi] = kr;
    }
  }
  if (tid == 0 && dropped != nullptr && s_drop != 0)
    atomicAdd(dropped, s_drop);
}

// Per-key totals of the count copies.
__global__ __launch_bounds__(256) void k_fold_copies(
    const uint32_t* __restrict__ copies, uint32_t nkeys,
    uint32_t* __restrict__ totals) {
  const uint32_t key = blockIdx.x * 256u + threadIdx.x;
  if (key >= nkeys) return;
  uint32_t c[kCountCopies];
#pragma unroll
  for (int x = 0; x < kCountCopies; ++x) c[x] = copies[(size_t)x * nkeys + key];
  uint32_t t = 0;
#pragma unroll
  for (int x = 0; x < kCountCopies; ++x) t += c[x];
  totals[key] = t;
}

// Copy x of key k becomes the offset of its first record: the key's offset
// plus the counts of the copies before x.
__global__ __launch_bounds__(256) void k_copy_offsets(
    uint32_t* __restrict__ copies, uint32_t nkeys,
    const uint32_t* __restrict__ offsets) {
  const uint32_t key = blockIdx.x * 256u + threadIdx.x;
  if (key >= nkeys) return;
  uint32_t c[kCountCopies];
#pragma unroll
  for (int x = 0; x < kCountCopies; ++x) c[x] = copies[(size_t)x * nkeys + key];
  uint32_t o = offsets[key];
#pragma unroll
  for (int x = 0; x < kCountCopies; ++x) {
    copies[(size_t)x * nkeys + key] = o;
    o += c[x];
  }
}

// ---- exclusive scan of uint32 counts (reduce, scan of block sums, apply) --

constexpr int kScanThreads = 256;
constexpr int kScanPerThread = 16;
constexpr int kScanBlock = kScanThreads * kScanPerThread;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v,
                                                         uint32_t* s_tmp,
                                                         uint32_t* total) {
  // Inclusive wave scan, then a scan of the wave totals.
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_tmp[wave] = x;
  __syncthreads();
  uint32_t wbase = 0;
  uint32_t all = 0;
  for (int w2 = 0; w2 < (int)(blockDim.x >> 6); ++w2) {
    const uint32_t t = s_tmp[w2];
    if (w2 < wave) wbase += t;
    all += t;
  }
  __syncthreads();
  *total = all;
  return wbase + x - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(
    const uint32_t* __restrict__ in, int64_t n, uint32_t* __restrict__ sums) {
  __shared__ uint32_t s_tmp[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  uint32_t acc = 0;
#pragma unroll
  for (int e = 0; e < kScanPerThread; ++e) {
    const int64_t i = base + (int64_t)e * kScanThreads + threadIdx.x;
    if (i < n) acc += in[i];
  }
  uint32_t total;
  block_exclusive_scan(acc, s_tmp, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_scan_sums(uint32_t* __restrict__ sums,
                                                    int64_t nb) {
  // One workgroup: exclusive scan of nb block sums in place; sums[nb] = total.
  __shared__ uint32_t s_tmp[16];
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += 1024) {
    const int64_t i = b0 + threadIdx.x;
    const uint32_t v = i < nb ? sums[i] : 0u;
    uint32_t total;
    const uint32_t ex = block_exclusive_scan(v, s_tmp, &total);
    if (i < nb) sums[i] = carry + ex;
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[nb] = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(
    const uint32_t* in, uint32_t* out, int64_t n,
    const uint32_t* __restrict__ sums, int64_t nb) {
  // Each thread owns kScanPerThread consecutive elements.
  __shared__ uint32_t s_tmp[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock +
                       (int64_t)threadIdx.x * kScanPerThread;
  uint32_t v[kScanPerThread];
  uint32_t acc = 0;
#pragma unroll
  for (int e = 0; e < kScanPerThread; ++e) {
    const int64_t i = base + e;
    v[e] = i < n ? in[i] : 0u;
    acc += v[e];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan(acc, s_tmp, &total) + sums[blockIdx.x];
#pragma unroll
  for (int e = 0; e < kScanPerThread; ++e) {
    const int64_t i = base + e;
    if (i < n) out[i] = run;
    run += v[e];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = sums[nb];
}

template <typename R>
__global__ __launch_bounds__(256) void k_bin_scatter(
    Geo g, VisSource src, int64_t m,
    const uint2* __restrict__ keyrank, const uint32_t* __restrict__ offsets,
    uint32_t nkeys, Record<R>* __restrict__ rec, int degrid,
    cplx<R>* __restrict__ vis_out) {
  const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= m) return;
  const uint2 kr = keyrank[gi];
  if (kr.x == kNoKey) {
    // No tap on the grid: no record, and a degridded value of zero (the
    // gather writes only the visibilities it has records for).
    if (degrid) vis_out[gi] = cplx<R>{(R)0, (R)0};
    return;
  }
  double x, y, u, v, w;
  int i0, j0, k;
  source_uvw(src, gi, u, v, w);
  place(g, u, v, w, x, y, i0, j0, k);
  // The copy the counting workgroup of this visibility added into.
  const int64_t copy = (gi / kCountPerBlock) % kCountCopies;
  const uint32_t pos = offsets[copy * nkeys + kr.x] + kr.y;
  Record<R> r;
  // Fractional offsets from the nearest cell, subtracted in FP64 first.
  r.dx = (R)(x - (double)i0);
  r.dy = (R)(y - (double)j0);
  if (!degrid) {
    const cplx<R> vv = source_value<R>(src, gi);
    r.vr = vv.re;
    r.vi = vv.im;
  } else {
    r.vr = (R)source_weight(src, gi);
    r.vi = (R)0;
  }
  r.cell = pack_cell(i0, j0);
  r.idx = (uint32_t)gi;
  rec[pos] = r;
}

// Appends to a list with one atomic per wavefront: returns this lane's slot
// (lanes with pred false get an unspecified value).
__device__ __forceinline__ uint32_t wave_append(uint32_t* counter, bool pred) {
  const unsigned long long mask = __ballot(pred);
  const int lane = threadIdx.x & 63;
  const int leader = mask ? (__ffsll((long long)mask) - 1) : 0;
  uint32_t base = 0;
  if (mask != 0 && lane == leader)
    base = atomicAdd(counter, (uint32_t)__popcll(mask));
  base = (uint32_t)__shfl((int)base, leader, 64);
  const unsigned long long below = mask & ((1ull << lane) - 1ull);
  return base + (uint32_t)__popcll(below);
}

__global__ __launch_bounds__(256) void k_tile_work(
    Geo g, const uint32_t* __restrict__ offsets, int mode_degrid,
    uint32_t chunk, uint32_t* __restrict__ tile_chunks,
    uint32_t* __restrict__ tile_slot, uint32_t* __restrict__ counters,
    uint32_t* __restrict__ split_list, uint32_t max_slots,
    uint2* __restrict__ extra, uint32_t max_extra,
    uint32_t* __restrict__ busy, uint32_t* __restrict__ idle,
    uint32_t* __restrict__ strips, uint32_t* __restrict__ tslot) {
  // counters[0]: scratch slots taken, [1]: split tiles, [2]: extra items,
  // [4]: tiles with records (listed in busy), [5]: tiles without (idle),
  // [6..7]: 64-bit sum of the records every tile reads.
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = t < g.ntiles;
  uint32_t work = 0;
  if (live) {
    if (mode_degrid) {
      work = offsets[(uint32_t)t * kRegions + kRegions] -
             offsets[(uint32_t)t * kRegions];
    } else {
      uint32_t lo[kSegments], hi[kSegments];
      tile_segments(g, t, lo, hi);
#pragma unroll
      for (int s = 0; s < kSegments; ++s)
        work += offsets[hi[s]] - offsets[lo[s]];
    }
  }
  // Busy tiles are listed per wavefront (the gridder takes items in list
  // order, and wavefront-sized runs of neighbouring tiles measured best);
  // idle tiles and the total record reads (diagnostics) need no order and
  // take one atomic per workgroup, which keeps same-address atomics, the
  // cost of this kernel, few.
  const uint32_t ib = wave_append(&counters[4], live && work > 0);
  __shared__ uint32_t s_idle[4];
  __shared__ unsigned long long s_reads[4];
  __shared__ uint32_t s_base;
  static_assert(4 * 64 == 256, "four wavefronts");
  const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
  const unsigned long long imask = __ballot(live && work == 0);
  unsigned long long wsum = work;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
    wsum += (unsigned long long)__shfl_xor((long long)wsum, o, 64);
  if (lane == 0) {
    s_idle[wave] = (uint32_t)__popcll(imask);
    s_reads[wave] = wsum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t n = s_idle[0] + s_idle[1] + s_idle[2] + s_idle[3];
    const unsigned long long reads =
        s_reads[0] + s_reads[1] + s_reads[2] + s_reads[3];
    s_base = n != 0 ? atomicAdd(&counters[5], n) : 0u;
    if (reads != 0)
      atomicAdd(reinterpret_cast<unsigned long long*>(&counters[6]), reads);
  }
  __syncthreads();
  uint32_t ii = s_base;
  for (int w = 0; w < wave; ++w) ii += s_idle[w];
  ii += (uint32_t)__popcll(imask & ((1ull << lane) - 1ull));
  if (!live) return;
  if (work > 0) {
    busy[ib] = (uint32_t)t;
    if (tslot != nullptr) tslot[t] = ib;  // its slot in the busy-tile store
  } else {
    idle[ii] = (uint32_t)t;
  }
  if (work > 0 && strips != nullptr) {
    // Column strip of this tile: plane k, tile column tx.
    const int per_plane = g.tiles_u * g.tiles_v;
    const int k = t / per_plane;
    const int tx = (t - k * per_plane) % g.tiles_u;
    strips[k * g.tiles_u + tx] = 1u;
  }
  uint32_t nch = work == 0 ? 1u : (work + chunk - 1) / chunk;
  tile_slot[t] = 0;
  if (nch > 1 && !mode_degrid) {
    const uint32_t s0 = atomicAdd(&counters[0], nch);
    if (s0 + nch <= max_slots) {
      tile_slot[t] = s0;
      split_list[atomicAdd(&counters[1], 1u)] = (uint32_t)t;
    } else {
      nch = 1;  // scratch exhausted: one item grids the whole tile
    }
  }
  if (nch > 1) {
    const uint32_t e0 = atomicAdd(&counters[2], nch - 1);
    if (e0 + (nch - 1) <= max_extra) {
      for (uint32_t c = 1; c < nch; ++c)
        extra[e0 + c - 1] = make_uint2((uint32_t)t, c);
    } else {
      nch = 1;  // cannot happen with the sizes the plan reserves
    }
  }
  // 0 marks a tile without records (its stack cells may be left unwritten
  // by a fused grid-and-image call).
  tile_chunks[t] = work == 0 ? 0u : nch;
}

// ---- two-level partition (no global atomics) ------------------------------
//
// Level 1 sorts the visibilities into coarse buckets (a plane and G rows of
// tiles: all the keys of one bucket are contiguous in key order), level 2
// sorts each bucket by its fine keys (tile column and region).  Both
// levels count in dense LDS histograms and publish one histogram per
// workgroup, so offsets come from scans, never from global atomics.  Both
// scatters first place their workgroup's records in LDS in output order
// (bucket by bucket, or key by key), then write them out as contiguous runs.
//
//   part_count1   placement, key, coarse bucket and the rank within the
//                 workgroup's bucket (LDS atomic); the workgroup's bucket
//                 histogram and its exclusive scan, block-major
//   col_*         bucket-major exclusive scan of the block-major
//                 histograms in place: offset of (bucket, block), and the
//                 bucket bounds
//   part_bounds   one workgroup: bucket bounds and the first level-2 chunk
//                 of every bucket (chunks of one staging area each)
//   part_scatter1 records built from the inputs, staged in LDS in bucket
//                 order, written to their bucket offsets, with their keys
//                 in a separate array (level 2 reads only the keys to
//                 count; the record's spare word carries the key through
//                 the staging)
//   part_count2   per chunk: fine key ranks (LDS atomic), the chunk's
//                 fine-key histogram and its exclusive scan
//   part_scan2    per bucket: chunk-major running sums of every fine key,
//                 the bucket's key offsets (the gridder's offsets table)
//   part_scatter2 records staged in LDS in key order, written to their
//                 key offsets
//
// Workgroups of level 1 and chunks of level 2 hold part_block<R>()
// visibilities: as many records as fit the LDS staging area.

constexpr int kPartThreads = 1024;
constexpr int kPartSegs = 64;  // block segments of the level-1 scan

// In-place exclusive scan of n LDS counters (each thread a contiguous run);
// returns the total.  Called by every thread of the workgroup.
__device__ __forceinline__ uint32_t lds_exclusive_scan(uint32_t* s, uint32_t n,
                                                       uint32_t* s_tmp) {
  const uint32_t per = (n + blockDim.x - 1) / blockDim.x;
  const uint32_t f0 = threadIdx.x * per;
  const uint32_t f1 = min(f0 + per, n);
  uint32_t acc = 0;
  for (uint32_t f = f0; f < f1; ++f) acc += s[f];
  uint32_t total;
  uint32_t run = block_exclusive_scan(acc, s_tmp, &total);
  for (uint32_t f = f0; f < f1; ++f) {
    const uint32_t v = s[f];
    s[f] = run;
    run += v;
  }
  __syncthreads();
  return total;
}

template <int V>
__global__ __launch_bounds__(kPartThreads) void k_part_count1(
    Geo g, VisSource src, int64_t m, uint32_t span, uint32_t nbuckets,
    uint2* __restrict__ keyrank, uint32_t* __restrict__ hist1,
    uint32_t* __restrict__ hist1x, uint32_t* __restrict__ btot,
    unsigned long long* __restrict__ dropped) {
  constexpr int PER = V / kPartThreads;
  extern __shared__ uint32_t s_h[];  // nbuckets counters
  __shared__ unsigned long long s_drop;
  __shared__ uint32_t s_tmp[kPartThreads / 64];
  const int tid = threadIdx.x;
  for (uint32_t c = tid; c < nbuckets; c += kPartThreads) s_h[c] = 0u;
  if (tid == 0) s_drop = 0;
  __syncthreads();
  unsigned long long my_drop = 0;
  const int64_t base = (int64_t)blockIdx.x * V;
  double cu[PER], cv[PER], cw[PER];
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    int64_t gi = base + (int64_t)e * kPartThreads + tid;
    gi = gi < m ? gi : m - 1;
    source_uvw(src, gi, cu[e], cv[e], cw[e]);
  }
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int64_t gi = base + (int64_t)e * kPartThreads + tid;
    if (gi >= m) continue;
    double x, y;
    int i0, j0, k;
    uint2 kr = make_uint2(kNoKey, 0u);
    if (place(g, cu[e], cv[e], cw[e], x, y, i0, j0, k)) {
      my_drop += (unsigned long long)(g.K * g.K - taps_on_grid(g, i0, j0));
      const uint32_t key = bin_key(g, i0, j0, k);
      kr.x = key;
      kr.y = atomicAdd(&s_h[key / span], 1u);
    } else {
      my_drop += (unsigned long long)(g.K * g.K);
    }
    keyrank[gi] = kr;
  }
  if (dropped != nullptr && my_drop != 0) atomicAdd(&s_drop, my_drop);
  __syncthreads();
  const size_t row = (size_t)blockIdx.x * nbuckets;
  for (uint32_t c = tid; c < nbuckets; c += kPartThreads)
    hist1[row + c] = s_h[c];
  __syncthreads();
  const uint32_t total = lds_exclusive_scan(s_h, nbuckets, s_tmp);
  for (uint32_t c = tid; c < nbuckets; c += kPartThreads)
    hist1x[row + c] = s_h[c];
  if (tid == 0) {
    btot[blockIdx.x] = total;
    if (dropped != nullptr && s_drop != 0) atomicAdd(dropped, s_drop);
  }
}

// Bucket-major exclusive scan of the block-major level-1 histograms
// (hist[b][c], b < nb blocks, c < nc buckets) without a transpose: the
// blocks are cut into nseg segments; col_sum totals each (segment,
// bucket), col_seg scans those over the segments and leaves each bucket's
// total, and col_apply turns the histograms into offsets in place:
//   hist[b][c] <- bounds[c] + sum over b' < b of hist[b'][c],
// bounds[c] the exclusive scan of the bucket totals (computed between
// col_seg and col_apply).
__global__ __launch_bounds__(256) void k_col_sum(
    const uint32_t* __restrict__ hist, uint32_t nb, uint32_t nc,
    uint32_t seglen, uint32_t* __restrict__ seg) {
  const uint32_t c = blockIdx.x * 256u + threadIdx.x;
  const uint32_t s = blockIdx.y;
  if (c >= nc) return;
  const uint32_t b0 = s * seglen, b1 = min(b0 + seglen, nb);
  uint32_t acc = 0;
  for (uint32_t b = b0; b < b1; ++b) acc += hist[(size_t)b * nc + c];
  seg[(size_t)s * nc + c] = acc;
}

__global__ __launch_bounds__(256) void k_col_seg(uint32_t* __restrict__ seg,
                                                 uint32_t nseg, uint32_t nc,
                                                 uint32_t* __restrict__ tot) {
  const uint32_t c = blockIdx.x * 256u + threadIdx.x;
  if (c >= nc) return;
  uint32_t run = 0;
  for (uint32_t s = 0; s < nseg; ++s) {
    const uint32_t v = seg[(size_t)s * nc + c];
    seg[(size_t)s * nc + c] = run;
    run += v;
  }
  tot[c] = run;
}

__global__ __launch_bounds__(256) void k_col_apply(
    uint32_t* __restrict__ hist, uint32_t nb, uint32_t nc, uint32_t seglen,
    const uint32_t* __restrict__ seg, const uint32_t* __restrict__ bounds) {
  const uint32_t c = blockIdx.x * 256u + threadIdx.x;
  const uint32_t s = blockIdx.y;
  if (c >= nc) return;
  const uint32_t b0 = s * seglen, b1 = min(b0 + seglen, nb);
  uint32_t run = bounds[c] + seg[(size_t)s * nc + c];
  // Eight loads in flight before the eight stores.
  uint32_t b = b0;
  for (; b + 8 <= b1; b += 8) {
    uint32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = hist[(size_t)(b + u) * nc + c];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      hist[(size_t)(b + u) * nc + c] = run;
      run += v[u];
    }
  }
  for (; b < b1; ++b) {
    uint32_t* p = hist + (size_t)b * nc + c;
    const uint32_t v = *p;
    *p = run;
    run += v;
  }
}

// offs1: the scanned (bucket, block) offsets, block-major (one row per
// workgroup); hist1x: the workgroup's own exclusive bucket offsets.
template <typename R, int V>
__global__ __launch_bounds__(kPartThreads) void k_part_scatter1(
    Geo g, VisSource src, int64_t m, const uint2* __restrict__ keyrank,
    const uint32_t* __restrict__ offs1, const uint32_t* __restrict__ hist1x,
    const uint32_t* __restrict__ btot, uint32_t span, uint32_t nbuckets,
    Record<R>* __restrict__ rec, uint32_t* __restrict__ keys, int degrid,
    cplx<R>* __restrict__ vis_out) {
  constexpr int PER = V / kPartThreads;
  extern __shared__ __align__(16) unsigned char s_raw[];
  Record<R>* s_rec = reinterpret_cast<Record<R>*>(s_raw);  // V records
  uint32_t* s_key = reinterpret_cast<uint32_t*>(s_rec + V);  // their keys
  const uint32_t b = blockIdx.x;
  const int64_t base = (int64_t)b * V;
  const uint32_t* ex = hist1x + (size_t)b * nbuckets;
  const uint32_t* off = offs1 + (size_t)b * nbuckets;
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int64_t gi = base + (int64_t)e * kPartThreads + threadIdx.x;
    if (gi >= m) continue;
    const uint2 kr = keyrank[gi];
    if (kr.x == kNoKey) {
      if (degrid) vis_out[gi] = cplx<R>{(R)0, (R)0};
      continue;
    }
    double x, y, u, v, w;
    int i0, j0, k;
    source_uvw(src, gi, u, v, w);
    place(g, u, v, w, x, y, i0, j0, k);
    Record<R> r;
    r.dx = (R)(x - (double)i0);
    r.dy = (R)(y - (double)j0);
    if (!degrid) {
      const cplx<R> vv = source_value<R>(src, gi);
      r.vr = vv.re;
      r.vi = vv.im;
    } else {
      r.vr = (R)source_weight(src, gi);
      r.vi = (R)0;
    }
    r.cell = pack_cell(i0, j0);
    r.idx = (uint32_t)gi;
    const uint32_t slot = ex[kr.x / span] + kr.y;
    s_rec[slot] = r;
    s_key[slot] = kr.x;  // for the write-out and level 2
  }
  __syncthreads();
  const uint32_t n = btot[b];
  for (uint32_t i = threadIdx.x; i < n; i += kPartThreads) {
    const uint32_t key = s_key[i];
    const uint32_t c = key / span;
    const uint32_t pos = off[c] + (i - ex[c]);
    rec[pos] = s_rec[i];
    keys[pos] = key;
  }
}

// One workgroup: bucket totals (in bounds[], from col_seg) -> bucket bounds
// (exclusive scan, bounds[nbuckets] = total), then chunks per bucket ->
// first chunk of every bucket (chunk0[nbuckets] = total chunks).  Each
// thread takes a contiguous run of buckets (nbuckets <= 16384).
__global__ __launch_bounds__(kPartThreads) void k_part_bounds(
    uint32_t* __restrict__ bounds, uint32_t nbuckets, uint32_t chunk,
    uint32_t* __restrict__ chunk0) {
  __shared__ uint32_t s_tmp[kPartThreads / 64];
  const uint32_t per = (nbuckets + kPartThreads - 1) / kPartThreads;
  const uint32_t c0 = threadIdx.x * per;
  const uint32_t c1 = min(c0 + per, nbuckets);
  uint32_t tot[16];
  uint32_t acc = 0;
  for (uint32_t c = c0; c < c1; ++c) {
    tot[c - c0] = bounds[c];
    acc += tot[c - c0];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan(acc, s_tmp, &total);
  uint32_t nch = 0;
  for (uint32_t c = c0; c < c1; ++c) {
    bounds[c] = run;
    run += tot[c - c0];
    nch += (tot[c - c0] + chunk - 1) / chunk;
  }
  uint32_t ntotal;
  uint32_t crun = block_exclusive_scan(nch, s_tmp, &ntotal);
  for (uint32_t c = c0; c < c1; ++c) {
    chunk0[c] = crun;
    crun += (tot[c - c0] + chunk - 1) / chunk;
  }
  if (threadIdx.x == 0) {
    bounds[nbuckets] = total;
    chunk0[nbuckets] = ntotal;
  }
}

// Bucket of chunk ch: the last c with chunk0[c] <= ch (chunk0 exclusive
// scan of the chunk counts, chunk0[nbuckets] = total), i.e. the bucket
// that owns the chunk even when empty buckets share its chunk0 value.
__device__ __forceinline__ uint32_t chunk_bucket(const uint32_t* chunk0,
                                                 uint32_t nbuckets,
                                                 uint32_t ch) {
  uint32_t lo = 0, hi = nbuckets;  // chunk0[lo] <= ch < chunk0[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (chunk0[mid] <= ch) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <int V>
__global__ __launch_bounds__(kPartThreads) void k_part_count2(
    const uint32_t* __restrict__ keys, const uint32_t* __restrict__ bounds,
    const uint32_t* __restrict__ chunk0, uint32_t nbuckets, uint32_t span,
    uint32_t* __restrict__ rank2, uint32_t* __restrict__ hist2,
    uint32_t* __restrict__ hist2x) {
  extern __shared__ uint32_t s_h[];  // span counters
  __shared__ uint32_t s_tmp[kPartThreads / 64];
  const uint32_t ch = blockIdx.x;
  if (ch >= chunk0[nbuckets]) return;
  const uint32_t c = chunk_bucket(chunk0, nbuckets, ch);
  const uint32_t start = bounds[c] + (ch - chunk0[c]) * V;
  const uint32_t end = min(start + (uint32_t)V, bounds[c + 1]);
  for (uint32_t f = threadIdx.x; f < span; f += kPartThreads) s_h[f] = 0u;
  __syncthreads();
  const uint32_t kb = c * span;
  for (uint32_t r = start + threadIdx.x; r < end; r += kPartThreads)
    rank2[r] = atomicAdd(&s_h[keys[r] - kb], 1u);
  __syncthreads();
  const size_t row = (size_t)ch * span;
  for (uint32_t f = threadIdx.x; f < span; f += kPartThreads)
    hist2[row + f] = s_h[f];
  __syncthreads();
  lds_exclusive_scan(s_h, span, s_tmp);
  for (uint32_t f = threadIdx.x; f < span; f += kPartThreads)
    hist2x[row + f] = s_h[f];
}

// One workgroup per bucket: hist2 of its chunks becomes the offset of
// every (chunk, fine key) share, and offsets[] of its keys is written.
__global__ __launch_bounds__(kPartThreads) void k_part_scan2(
    const uint32_t* __restrict__ bounds, const uint32_t* __restrict__ chunk0,
    uint32_t nbuckets, uint32_t span, uint32_t* __restrict__ hist2,
    uint32_t* __restrict__ offsets) {
  extern __shared__ uint32_t s_tot[];  // span totals
  __shared__ uint32_t s_tmp[kPartThreads / 64];
  const uint32_t c = blockIdx.x;
  const uint32_t base = bounds[c];
  const uint32_t q0 = chunk0[c], q1 = chunk0[c + 1];
  for (uint32_t f = threadIdx.x; f < span; f += kPartThreads) {
    uint32_t run = 0;
    uint32_t q = q0;
    for (; q + 8 <= q1; q += 8) {  // eight loads in flight, then the stores
      uint32_t v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = hist2[(size_t)(q + u) * span + f];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        hist2[(size_t)(q + u) * span + f] = run;
        run += v[u];
      }
    }
    for (; q < q1; ++q) {
      uint32_t* p = hist2 + (size_t)q * span + f;
      const uint32_t v = *p;
      *p = run;
      run += v;
    }
    s_tot[f] = run;
  }
  __syncthreads();
  lds_exclusive_scan(s_tot, span, s_tmp);
  for (uint32_t f = threadIdx.x; f < span; f += kPartThreads) {
    const uint32_t o = base + s_tot[f];
    offsets[(size_t)c * span + f] = o;
    for (uint32_t q = q0; q < q1; ++q) hist2[(size_t)q * span + f] += o;
  }
  if (c + 1 == nbuckets && threadIdx.x == 0)
    offsets[(size_t)nbuckets * span] = bounds[nbuckets];
}

template <typename R, int V>
__global__ __launch_bounds__(kPartThreads) void k_part_scatter2(
    const uint32_t* __restrict__ keys, const uint32_t* __restrict__ bounds,
    const uint32_t* __restrict__ chunk0, uint32_t nbuckets, uint32_t span,
    const uint32_t* __restrict__ rank2, const uint32_t* __restrict__ hist2,
    const uint32_t* __restrict__ hist2x,
    const Record<R>* __restrict__ rec1, Record<R>* __restrict__ rec) {
  extern __shared__ __align__(16) unsigned char s_raw[];
  Record<R>* s_rec = reinterpret_cast<Record<R>*>(s_raw);  // V records
  uint32_t* s_fine = reinterpret_cast<uint32_t*>(s_rec + V);  // fine keys
  const uint32_t ch = blockIdx.x;
  if (ch >= chunk0[nbuckets]) return;
  const uint32_t c = chunk_bucket(chunk0, nbuckets, ch);
  const uint32_t start = bounds[c] + (ch - chunk0[c]) * V;
  const uint32_t end = min(start + (uint32_t)V, bounds[c + 1]);
  const uint32_t* off = hist2 + (size_t)ch * span;
  const uint32_t* ex = hist2x + (size_t)ch * span;
  const uint32_t kb = c * span;
  for (uint32_t r = start + threadIdx.x; r < end; r += kPartThreads) {
    const uint32_t f = keys[r] - kb;
    const uint32_t slot = ex[f] + rank2[r];
    s_rec[slot] = rec1[r];
    s_fine[slot] = f;
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < end - start; i += kPartThreads) {
    const uint32_t f = s_fine[i];
    rec[off[f] + (i - ex[f])] = s_rec[i];
  }
}

}  // namespace

// Two-level partition of m visibilities (see the kernels above), in the
// phases the library times separately.
namespace {
template <typename R>
constexpr int part_block() {
  // LDS staging of one workgroup: 4096 24-byte (FP32) or 2048 40-byte
  // (FP64) records and their keys.
  return sizeof(R) == 4 ? 4096 : 2048;
}
int part_block_of(int elem) { return elem == 8 ? 4096 : 2048; }
uint32_t part_nb1(int64_t m, int V) {
  const int64_t nb = (m + V - 1) / V;
  return (uint32_t)(nb > 0 ? nb : 1);
}
uint32_t part_max_chunks(int64_t m, uint32_t nbuckets, int V) {
  return (uint32_t)((m + V - 1) / V) + nbuckets;
}
}  // namespace

template <typename R>
void launch_part_count1(const Geo& g, const VisSource& src, int64_t m,
                        const PartWork& w, unsigned long long* dropped,
                        hipStream_t st) {
  if (m == 0) return;
  constexpr int V = part_block<R>();
  hipLaunchKernelGGL(k_part_count1<V>, dim3(part_nb1(m, V)),
                     dim3(kPartThreads), (size_t)w.nbuckets * 4, st, g, src, m,
                     w.span, w.nbuckets, w.keyrank, w.hist1, w.hist1x, w.btot,
                     dropped);
}

template <typename R>
void launch_part_scan1(int64_t m, const PartWork& w, hipStream_t st) {
  constexpr int V = part_block<R>();
  const uint32_t C = w.nbuckets;
  const dim3 cg((C + 255) / 256);
  if (m > 0) {
    const uint32_t nb1 = part_nb1(m, V);
    const uint32_t nseg = nb1 < (uint32_t)kPartSegs ? nb1 : (uint32_t)kPartSegs;
    const uint32_t seglen = (nb1 + nseg - 1) / nseg;
    hipLaunchKernelGGL(k_col_sum, dim3(cg.x, nseg), dim3(256), 0, st,
                       w.hist1, nb1, C, seglen, w.seg);
    hipLaunchKernelGGL(k_col_seg, cg, dim3(256), 0, st, w.seg, nseg, C,
                       w.bounds);
  } else {
    launch_zero_u32(w.bounds, (int64_t)C + 1, st);
  }
  hipLaunchKernelGGL(k_part_bounds, dim3(1), dim3(kPartThreads), 0, st,
                     w.bounds, C, (uint32_t)V, w.chunk0);
  if (m > 0) {
    const uint32_t nb1 = part_nb1(m, V);
    const uint32_t nseg = nb1 < (uint32_t)kPartSegs ? nb1 : (uint32_t)kPartSegs;
    const uint32_t seglen = (nb1 + nseg - 1) / nseg;
    hipLaunchKernelGGL(k_col_apply, dim3(cg.x, nseg), dim3(256), 0, st,
                       w.hist1, nb1, C, seglen, w.seg, w.bounds);
  }
}

template <typename R>
void launch_part_scatter1(const Geo& g, const VisSource& src, int64_t m,
                          const PartWork& w, int degrid, void* vis_out,
                          hipStream_t st) {
  if (m == 0) return;
  constexpr int V = part_block<R>();
  hipLaunchKernelGGL((k_part_scatter1<R, V>), dim3(part_nb1(m, V)),
                     dim3(kPartThreads), (size_t)V * (sizeof(Record<R>) + 4),
                     st, g, src, m, w.keyrank, w.hist1, w.hist1x, w.btot,
                     w.span, w.nbuckets, (Record<R>*)w.rec1, w.keys, degrid,
                     (cplx<R>*)vis_out);
}

template <typename R>
void launch_part_count2(int64_t m, const PartWork& w, hipStream_t st) {
  if (m == 0) return;
  constexpr int V = part_block<R>();
  hipLaunchKernelGGL(k_part_count2<V>,
                     dim3(part_max_chunks(m, w.nbuckets, V)),
                     dim3(kPartThreads), (size_t)w.span * 4, st, w.keys,
                     w.bounds, w.chunk0, w.nbuckets, w.span, w.rank2, w.hist2,
                     w.hist2x);
}

template <typename R>
void launch_part_scan2(int64_t, const PartWork& w, hipStream_t st) {
  hipLaunchKernelGGL(k_part_scan2, dim3(w.nbuckets), dim3(kPartThreads),
                     (size_t)w.span * 4, st, w.bounds, w.chunk0, w.nbuckets,
                     w.span, w.hist2, w.offsets);
}

template <typename R>
void launch_part_scatter2(int64_t m, const PartWork& w, hipStream_t st) {
  if (m == 0) return;
  constexpr int V = part_block<R>();
  hipLaunchKernelGGL((k_part_scatter2<R, V>),
                     dim3(part_max_chunks(m, w.nbuckets, V)),
                     dim3(kPartThreads), (size_t)V * (sizeof(Record<R>) + 4),
                     st, w.keys, w.bounds, w.chunk0, w.nbuckets, w.span, w.rank2,
                     w.hist2, w.hist2x, (const Record<R>*)w.rec1,
                     (Record<R>*)w.rec);
}

#define WS_INST(R)                                                           \
  template void launch_part_count1<R>(const Geo&, const VisSource&, int64_t, \
                                      const PartWork&, unsigned long long*, \
                                      hipStream_t);                         \
  template void launch_part_scan1<R>(int64_t, const PartWork&, hipStream_t); \
  template void launch_part_scatter1<R>(const Geo&, const VisSource&,       \
                                        int64_t, const PartWork&, int,      \
                                        void*, hipStream_t);                \
  template void launch_part_count2<R>(int64_t, const PartWork&,             \
                                      hipStream_t);                         \
  template void launch_part_scan2<R>(int64_t, const PartWork&, hipStream_t); \
  template void launch_part_scatter2<R>(int64_t, const PartWork&,           \
                                        hipStream_t);
WS_INST(float)
WS_INST(double)
#undef WS_INST

int64_t partition_blocks(int64_t max_vis, int elem) {
  const int V = part_block_of(elem);
  return (max_vis + V - 1) / V;
}
int64_t partition_chunks(int64_t max_vis, int64_t nbuckets, int elem) {
  const int V = part_block_of(elem);
  return (max_vis + V - 1) / V + nbuckets;
}

void launch_bin_count(const Geo& g, const VisSource& src, int64_t m,
                      uint32_t* copies, uint32_t nkeys, uint2* keyrank,
                      unsigned long long* dropped, hipStream_t st) {
  if (m == 0) return;
  const int64_t nb = (m + kCountPerBlock - 1) / kCountPerBlock;
  hipLaunchKernelGGL(k_bin_count, dim3((unsigned)nb), dim3(kCountThreads), 0,
                     st, g, src, m, copies, nkeys, keyrank, dropped);
}

void launch_fold_copies(const uint32_t* copies, uint32_t nkeys,
                        uint32_t* totals, hipStream_t st) {
  hipLaunchKernelGGL(k_fold_copies, dim3((nkeys + 255) / 256), dim3(256), 0,
                     st, copies, nkeys, totals);
}

void launch_copy_offsets(uint32_t* copies, uint32_t nkeys,
                         const uint32_t* offsets, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_offsets, dim3((nkeys + 255) / 256), dim3(256), 0,
                     st, copies, nkeys, offsets);
}

int64_t scan_sums_len(int64_t n) { return (n + kScanBlock - 1) / kScanBlock + 1; }

void launch_exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n,
                           uint32_t* sums, hipStream_t st) {
  // out has n + 1 entries; out[n] = total.  in may alias out.
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0,
                     st, in, n, sums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, st, sums, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0,
                     st, in, out, n, sums, nb);
}

template <typename R>
void launch_bin_scatter(const Geo& g, const VisSource& src, int64_t m,
                        const uint2* keyrank, const uint32_t* offsets,
                        uint32_t nkeys, void* records, int degrid,
                        void* vis_out, hipStream_t st) {
  if (m == 0) return;
  const int64_t nb = (m + 255) / 256;
  hipLaunchKernelGGL(k_bin_scatter<R>, dim3((unsigned)nb), dim3(256), 0, st, g,
                     src, m, keyrank, offsets, nkeys, (Record<R>*)records,
                     degrid, (cplx<R>*)vis_out);
}

template void launch_bin_scatter<float>(const Geo&, const VisSource&, int64_t,
                                        const uint2*, const uint32_t*,
                                        uint32_t, void*, int, void*,
                                        hipStream_t);
template void launch_bin_scatter<double>(const Geo&, const VisSource&,
                                         int64_t, const uint2*,
                                         const uint32_t*, uint32_t, void*,
                                         int, void*, hipStream_t);

void launch_tile_work(const Geo& g, const uint32_t* offsets, int mode_degrid,
                      uint32_t chunk, uint32_t* tile_chunks,
                      uint32_t* tile_slot, uint32_t* counters,
                      uint32_t* split_list, uint32_t max_slots, uint2* extra,
                      uint32_t max_extra, uint32_t* busy, uint32_t* idle,
                      uint32_t* strips, uint32_t* tslot, hipStream_t st) {
  const int nb = (g.ntiles + 255) / 256;
  hipLaunchKernelGGL(k_tile_work, dim3(nb), dim3(256), 0, st, g, offsets,
                     mode_degrid, chunk, tile_chunks, tile_slot, counters,
                     split_list, max_slots, extra, max_extra, busy, idle,
                     strips, tslot);
}

}  // namespace ws
