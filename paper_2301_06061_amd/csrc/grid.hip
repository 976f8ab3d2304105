// Gridding (Eq. 3) and degridding (its adjoint) over binned records.
//
// Gridding: persistent workgroups (as many as fit on the device) take work
// items from a queue in device memory.  A tile lives in LDS as separate
// real and imaginary rows of FP64 accumulators on both precision paths: on
// this part LDS FP64 atomic adds run about 20x faster than FP32 ones
// (measured, 6.6 vs 0.33 lanes per clock per CU), so the FP32 path computes
// its taps in FP32 and sums them in FP64 before rounding the finished tile
// to FP32.  A wavefront takes one visibility at a time and its lanes cover
// the K x K kernel taps, so the adds of one LDS instruction hit distinct
// cells (no same-address serialisation, even in a dense core where many
// visibilities share a cell); the LDS row pitch is T + K (odd), so they
// also fall in distinct banks.
//
// Latency hiding: the records of a tile come from up to ten key ranges
// (its own bins and its neighbours' edge strips); they are read as one
// concatenated list, 64 per wavefront and all wavefronts at once, with the
// next batch loaded while the current one is accumulated.  The next work
// item is taken from the queue, and its key ranges are loaded, while the
// current tile is written out; writing a tile also clears its LDS, so no
// separate clearing pass is needed.
//
// A tile is written to HBM once, zeros included, with 16-byte row stores;
// tiles with more records than one chunk are split over several items
// whose partial tiles a merge kernel sums in a fixed order.  The queue
// hands out the extra chunks of split (hot) tiles first, then one item per
// tile with records, then groups of tiles without records, which only get
// zeros.
//
// Degridding: persistent workgroups take (tile, chunk) items; each loads
// the transformed plane's tile plus an h-cell halo into LDS once, and each
// lane evaluates one visibility's K x K weighted sum from LDS.
#include "ws_kernels.h"

namespace ws {

namespace {

constexpr int kGridThreads = 512;

// Workgroup barrier that orders LDS only.  The persistent kernels below
// never read, within one launch, global memory that another workgroup
// writes, so their barriers need not wait for outstanding global stores:
// a tile's stores drain while the workgroup goes on to the next item.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// One-dimensional kernel factor g(d) = exp(-d^2 / (2 sigma^2)); FP32 uses
// the hardware base-2 exponential (v_exp_f32) with a pre-scaled argument.
// Arguments never approach the denormal range that would need rescaling:
// the farthest tap of the widest kernel is at 2^-30 or above.
__device__ __forceinline__ float gauss1(const Geo& g, float d) {
  return __builtin_amdgcn_exp2f(-g.kappa * (d * d));
}
__device__ __forceinline__ double gauss1(const Geo& g, double d) {
  return exp(-g.inv2s2 * (d * d));
}

// Two-dimensional tap weight g(dx) g(dy) = exp(-(dx^2 + dy^2)/(2 sigma^2))
// from the squared distance: one exponential per tap.
__device__ __forceinline__ float gauss2(const Geo& g, float d2) {
  return __builtin_amdgcn_exp2f(-g.kappa * d2);
}
__device__ __forceinline__ double gauss2(const Geo& g, double d2) {
  return exp(-g.inv2s2 * d2);
}

// Idle tiles are zeroed kZeroGroup to a work item.
constexpr int kZeroGroup = 8;

struct Item {
  int zero;        // 1: a group of idle tiles to zero
  int tile;
  uint32_t chunk;  // chunk of the tile, or the group index
};

__device__ __forceinline__ uint32_t item_total(const uint32_t* counters,
                                               bool with_zero) {
  const uint32_t n = counters[2] + counters[4];
  return with_zero ? n + (counters[5] + kZeroGroup - 1) / kZeroGroup : n;
}

__device__ __forceinline__ Item resolve_item(uint32_t item,
                                             const uint32_t* counters,
                                             const uint2* extra,
                                             const uint32_t* busy) {
  const uint32_t nextra = counters[2], nbusy = counters[4];
  Item it;
  if (item < nextra) {
    const uint2 tc = extra[item];
    it.zero = 0;
    it.tile = (int)tc.x;
    it.chunk = tc.y;
  } else if (item < nextra + nbusy) {
    it.zero = 0;
    it.tile = (int)busy[item - nextra];
    it.chunk = 0;
  } else {
    it.zero = 1;
    it.tile = 0;
    it.chunk = item - nextra - nbusy;
  }
  return it;
}

// Pop the next item of a plan's own queue (counters[3]); used by the
// degridder.  Contains the barriers that order LDS reuse between items.
__device__ __forceinline__ bool next_item(const uint32_t* counters_ro,
                                          uint32_t* counters,
                                          const uint2* extra,
                                          const uint32_t* busy, bool with_zero,
                                          uint32_t* s_item, Item& it) {
  lds_barrier();
  if (threadIdx.x == 0) *s_item = atomicAdd(&counters[3], 1u);
  lds_barrier();
  const uint32_t item = *s_item;
  if (item >= item_total(counters_ro, with_zero)) return false;
  it = resolve_item(item, counters_ro, extra, busy);
  return true;
}

__device__ __forceinline__ void tile_origin(const Geo& g, int t, int& k,
                                            int& oy, int& ox) {
  const int per_plane = g.tiles_u * g.tiles_v;
  k = t / per_plane;
  const int rem = t - k * per_plane;
  oy = (rem / g.tiles_u) * g.T;
  ox = (rem % g.tiles_u) * g.T;
}

__device__ __forceinline__ void store16(cplx<float>* p, const cplx<float>* v) {
  *reinterpret_cast<float4*>(p) = make_float4(v[0].re, v[0].im, v[1].re,
                                              v[1].im);
}
__device__ __forceinline__ void store16(cplx<double>* p,
                                        const cplx<double>* v) {
  *p = v[0];
}

// Store (or add) a T x T tile of FP64 LDS accumulators, held as separate
// real and imaginary rows, into a row-major complex destination of the
// path precision, 16 bytes per store; the LDS cells read are cleared.
template <typename R>
__device__ __forceinline__ void store_tile_clear(double* s_re, double* s_im,
                                                 int pitch, int T,
                                                 double scale, cplx<R>* dst,
                                                 size_t dst_pitch,
                                                 bool accumulate) {
  constexpr int V = 16 / sizeof(cplx<R>);  // complex values per store
  const int per_row = T / V;
  for (int i = threadIdx.x; i < T * per_row; i += blockDim.x) {
    const int lj = i / per_row, li = (i - lj * per_row) * V;
    cplx<R> v[V];
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const int a = lj * pitch + li + e;
      v[e] = {(R)(scale * s_re[a]), (R)(scale * s_im[a])};
      s_re[a] = 0.0;
      s_im[a] = 0.0;
    }
    cplx<R>* p = dst + (size_t)lj * dst_pitch + li;
    if (accumulate) {
#pragma unroll
      for (int e = 0; e < V; ++e) v[e] = cadd(p[e], v[e]);
    }
    store16(p, v);
  }
}

template <typename R>
__device__ __forceinline__ void zero_tile(int T, cplx<R>* dst,
                                          size_t dst_pitch) {
  constexpr int V = 16 / sizeof(cplx<R>);
  const int per_row = T / V;
  for (int i = threadIdx.x; i < T * per_row; i += blockDim.x) {
    const int lj = i / per_row, li = (i - lj * per_row) * V;
    *reinterpret_cast<float4*>(dst + (size_t)lj * dst_pitch + li) =
        make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

template <typename R>
__device__ __forceinline__ R bcast(R x, int lane);
template <>
__device__ __forceinline__ float bcast<float>(float x, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}
template <>
__device__ __forceinline__ double bcast<double>(double x, int lane) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFFll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) |
                              (long long)(unsigned)lo);
}
__device__ __forceinline__ uint32_t bcast_u(uint32_t x, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, lane);
}
__device__ __forceinline__ uint32_t uniform(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

// A work item resolved for gridding (the same in every thread).  The
// records of a tile are the concatenation of its key ranges; position f of
// that list is record f + off0 + the sum of step[s] over the ranges s >= 1
// with cum[s] <= f.  The item covers positions [f0, f1).
struct GridItem {
  int valid;
  int zero;
  int tile;        // tile index, or the zero group index
  uint32_t nch;    // items the tile is split into
  uint32_t chunk;  // which of them
  uint32_t f0, f1;
  uint32_t off0;
  uint32_t cum[kSegments];
  uint32_t step[kSegments];
};

// Loads are unconditional (with indices that are valid whatever the item)
// and results are selected afterwards, so that the compiler issues them
// back to back instead of one guarded load and wait at a time.
template <typename R>
__device__ __forceinline__ GridItem prepare_item(const GridJob<R>& j,
                                                 uint32_t local,
                                                 uint32_t nextra,
                                                 uint32_t nbusy,
                                                 uint32_t total) {
  GridItem x;
  x.valid = local < total;
  x.zero = local >= nextra + nbusy;
  const bool is_extra = local < nextra;
  const bool live = x.valid && !x.zero;
  // First level: which tile (and chunk) the item is.
  const uint2 tc = j.extra[is_extra ? local : 0u];
  const uint32_t bt = j.busy[live && !is_extra ? local - nextra : 0u];
  uint32_t tile = is_extra ? tc.x : bt;
  x.chunk = uniform(is_extra ? tc.y : 0u);
  if (!live) tile = 0;
  x.tile = (int)uniform(tile);
  // Second level: the tile's split count and key ranges.
  const uint32_t nch = j.tile_chunks[x.tile];
  uint32_t lo[kSegments], hi[kSegments], a[kSegments], b[kSegments];
  tile_segments(j.g, x.tile, lo, hi);
#pragma unroll
  for (int s = 0; s < kSegments; ++s) {
    a[s] = j.offsets[lo[s]];
    b[s] = j.offsets[hi[s]];
  }
  x.nch = live ? uniform(nch) : 1u;
  uint32_t cum = 0, prev = 0;
#pragma unroll
  for (int s = 0; s < kSegments; ++s) {
    const uint32_t as = live ? uniform(a[s]) : 0u;
    const uint32_t bs = live ? uniform(b[s]) : 0u;
    const uint32_t off = as - cum;
    x.cum[s] = cum;
    x.step[s] = off - prev;
    if (s == 0) x.off0 = off;
    prev = off;
    cum += bs - as;
  }
  if (x.valid && x.zero) x.tile = (int)(local - nextra - nbusy);
  x.f0 = x.chunk * j.chunk;
  x.f1 = x.nch == 1 ? cum : min(cum, x.f0 + j.chunk);
  return x;
}

// Record index of list position f of item x (a sum of selects, so that
// the per-range values stay in registers).
__device__ __forceinline__ uint32_t record_at(const GridItem& x, uint32_t f) {
  uint32_t r = f + x.off0;
#pragma unroll
  for (int s = 1; s < kSegments; ++s) r += f >= x.cum[s] ? x.step[s] : 0u;
  return r;
}

template <typename R>
struct RecBatch {
  uint32_t cell;
  cplx<R> dxy, val;
};

// Loads list position f of the item; positions past the end re-read the
// last record (so the loads need no branch) and give a zero value.
template <typename R>
__device__ __forceinline__ RecBatch<R> load_batch(const GridJob<R>& j,
                                                  const GridItem& x,
                                                  uint32_t f) {
  const bool in = f < x.f1;
  const uint32_t r = record_at(x, in ? f : x.f1 - 1);
  RecBatch<R> b;
  b.cell = j.rec_cell[r];
  b.dxy = j.rec_dxy[r];
  b.val = j.rec_val[r];
  if (!in) b.val = {(R)0, (R)0};
  return b;
}

// Accumulates the item's records into the LDS tile.  Every wavefront takes
// batches of 64 list positions, strided by the workgroup; the next batch
// is in flight while the current one is added.
template <typename R, int K>
__device__ __forceinline__ void accumulate_item(const GridJob<R>& j,
                                                const GridItem& x,
                                                double* s_re, double* s_im) {
  constexpr int H = (K - 1) / 2;
  constexpr int KK = K * K;
  constexpr int ROUNDS = (KK + 63) / 64;
  const int T = j.g.T;
  const int pitch = j.pitch;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const uint32_t step = (uint32_t)(blockDim.x >> 6) * 64u;
  int k, oy, ox;
  tile_origin(j.g, x.tile, k, oy, ox);
  int ta[ROUNDS], tb[ROUNDS], toff[ROUNDS];
#pragma unroll
  for (int q = 0; q < ROUNDS; ++q) {
    const int tt = lane + 64 * q;
    ta[q] = tt % K - H;
    tb[q] = tt / K - H;
    toff[q] = tb[q] * pitch + ta[q];
  }
  uint32_t b0 = x.f0 + (uint32_t)wave * 64u;
  RecBatch<R> cur = load_batch(j, x, b0 + lane);
  while (b0 < x.f1) {
    const uint32_t b1 = b0 + step;
    const RecBatch<R> nxt = load_batch(j, x, b1 + lane);
    const int cnt = (x.f1 - b0) < 64u ? (int)(x.f1 - b0) : 64;
    for (int r = 0; r < cnt; ++r) {
      const uint32_t cc = bcast_u(cur.cell, r);
      const R dx = bcast(cur.dxy.re, r), dy = bcast(cur.dxy.im, r);
      const R vr = bcast(cur.val.re, r), vi = bcast(cur.val.im, r);
      const int ci = cell_i(cc) - ox, cj = cell_j(cc) - oy;
      const int base = cj * pitch + ci;
#pragma unroll
      for (int q = 0; q < ROUNDS; ++q) {
        if (KK % 64 == 0 || lane + 64 * q < KK) {
          const int li = ci + ta[q], lj = cj + tb[q];
          if ((unsigned)li < (unsigned)T && (unsigned)lj < (unsigned)T) {
            const R ex = (R)ta[q] - dx, ey = (R)tb[q] - dy;
            const R w = gauss2(j.g, ex * ex + ey * ey);
            atomicAdd(s_re + base + toff[q], (double)(w * vr));
            atomicAdd(s_im + base + toff[q], (double)(w * vi));
          }
        }
      }
    }
    cur = nxt;
    b0 = b1;
  }
}

// Writes a finished item: the whole tile (scaled by the kernel norm), or
// one partial tile of a split tile.  Clears the LDS cells it reads.
template <typename R>
__device__ __forceinline__ void store_item(const GridJob<R>& j,
                                           const GridItem& x, double* s_re,
                                           double* s_im) {
  const int T = j.g.T;
  if (x.nch == 1) {
    int k, oy, ox;
    tile_origin(j.g, x.tile, k, oy, ox);
    cplx<R>* dst = j.planes + ((size_t)k * j.g.nv + oy) * j.g.nu + ox;
    store_tile_clear(s_re, s_im, j.pitch, T, j.g.cnorm, dst,
                     (size_t)j.g.nu, j.accumulate != 0);
  } else {
    cplx<R>* part =
        j.partials + (size_t)(j.tile_slot[x.tile] + x.chunk) * T * T;
    store_tile_clear(s_re, s_im, j.pitch, T, 1.0, part, (size_t)T, false);
  }
}

template <typename R>
__device__ __forceinline__ void zero_group(const GridJob<R>& j, int group) {
  const uint32_t nidle = j.counters[5];
  const uint32_t z0 = (uint32_t)group * kZeroGroup;
  // All tile numbers first (unconditional loads of valid entries), so
  // that their loads overlap.
  uint32_t t[kZeroGroup];
#pragma unroll
  for (int z = 0; z < kZeroGroup; ++z) {
    const uint32_t v = j.idle[z0 + z < nidle ? z0 + z : 0u];
    t[z] = z0 + z < nidle ? uniform(v) : 0xFFFFFFFFu;
  }
#pragma unroll
  for (int z = 0; z < kZeroGroup; ++z) {
    if (t[z] == 0xFFFFFFFFu) continue;
    int k, oy, ox;
    tile_origin(j.g, (int)t[z], k, oy, ox);
    zero_tile(j.g.T, j.planes + ((size_t)k * j.g.nv + oy) * j.g.nu + ox,
              (size_t)j.g.nu);
  }
}

__device__ __forceinline__ void clear_lds(double* s, uint32_t words) {
  for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) s[i] = 0.0;
}

// The first half of a work item: zero a group of idle tiles, or add the
// item's records into the LDS tile (written out after the next barrier).
template <typename R, int K>
__device__ __forceinline__ void do_item(const GridJob<R>& j, const GridItem& x,
                                        double* s_re, double* s_im) {
  if (x.zero) {
    zero_group(j, x.tile);
    return;
  }
  if (x.f1 > x.f0) accumulate_item<R, K>(j, x, s_re, s_im);
}

template <typename R, int K>
__global__ __launch_bounds__(kGridThreads) void k_grid_tiles(GridJob<R> j) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t s_next;
  double* s_re = reinterpret_cast<double*>(smem);
  double* s_im = s_re + j.g.T * j.pitch;
  const bool with_zero = !j.accumulate;
  const uint32_t nextra = j.counters[2], nbusy = j.counters[4];
  const uint32_t total = item_total(j.counters, with_zero);
  uint32_t* queue = &j.counters[3];
  clear_lds(s_re, 2u * (uint32_t)(j.g.T * j.pitch));
  if (threadIdx.x == 0) s_next = atomicAdd(queue, 1u);
  lds_barrier();
  GridItem x = prepare_item(j, uniform(s_next), nextra, nbusy, total);
  while (x.valid) {
    lds_barrier();  // every thread has read s_next
    if (threadIdx.x == 0) s_next = atomicAdd(queue, 1u);
    do_item<R, K>(j, x, s_re, s_im);
    lds_barrier();  // LDS sums complete; s_next visible
    const GridItem nx = prepare_item(j, uniform(s_next), nextra, nbusy, total);
    if (!x.zero) {
      if (x.f1 > x.f0)
        store_item(j, x, s_re, s_im);
      else if (x.nch == 1 && !j.accumulate) {
        int k, oy, ox;
        tile_origin(j.g, x.tile, k, oy, ox);
        zero_tile(j.g.T, j.planes + ((size_t)k * j.g.nv + oy) * j.g.nu + ox,
                  (size_t)j.g.nu);
      }
    }
    x = nx;
  }
}

// Batched gridding: one persistent launch drains a single queue holding the
// work items of every job (plan), job after job; the LDS tile is sized for
// the largest tile of the batch (lds_words FP64 words in all).
template <typename R, int K>
__global__ __launch_bounds__(kGridThreads) void k_grid_batch(
    const GridJob<R>* __restrict__ jobs, int njobs,
    uint32_t* __restrict__ queue, uint32_t lds_words) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t s_next;
  __shared__ uint32_t s_base[kMaxBatch + 1];
  double* s_re = reinterpret_cast<double*>(smem);
  if (threadIdx.x == 0) {
    uint32_t b = 0;
    for (int p = 0; p < njobs; ++p) {
      s_base[p] = b;
      b += item_total(jobs[p].counters, !jobs[p].accumulate);
    }
    s_base[njobs] = b;
    s_next = atomicAdd(queue, 1u);
  }
  clear_lds(s_re, lds_words);
  lds_barrier();
  // Resolve a queue number to (job, item of that job); jobs are read in
  // place (uniform loads), never copied.
  auto resolve = [&](uint32_t item, int& p) -> GridItem {
    item = uniform(item);
    p = 0;
    const bool live = item < s_base[njobs];
    if (live)
      while (item >= s_base[p + 1]) ++p;
    const GridJob<R>& jj = jobs[p];
    const uint32_t total = live ? item_total(jj.counters, !jj.accumulate) : 0u;
    return prepare_item(jj, live ? item - s_base[p] : 0u, jj.counters[2],
                        jj.counters[4], total);
  };
  int p = 0;
  GridItem x = resolve(s_next, p);
  while (x.valid) {
    lds_barrier();
    if (threadIdx.x == 0) s_next = atomicAdd(queue, 1u);
    const GridJob<R>& j = jobs[p];
    double* s_im = s_re + j.g.T * j.pitch;
    do_item<R, K>(j, x, s_re, s_im);
    lds_barrier();
    int pn = 0;
    const GridItem nx = resolve(s_next, pn);
    if (!x.zero) {
      if (x.f1 > x.f0)
        store_item(j, x, s_re, s_im);
      else if (x.nch == 1 && !j.accumulate) {
        int k, oy, ox;
        tile_origin(j.g, x.tile, k, oy, ox);
        zero_tile(j.g.T, j.planes + ((size_t)k * j.g.nv + oy) * j.g.nu + ox,
                  (size_t)j.g.nu);
      }
    }
    x = nx;
    p = pn;
  }
}

template <typename R>
__global__ __launch_bounds__(1024) void k_grid_merge(
    Geo g, const uint32_t* __restrict__ counters,
    const uint32_t* __restrict__ split_list,
    const uint32_t* __restrict__ tile_chunks,
    const uint32_t* __restrict__ tile_slot,
    const cplx<R>* __restrict__ partials, cplx<R>* __restrict__ planes,
    int accumulate) {
  // One workgroup per split tile sums its partial tiles in chunk order.
  if (blockIdx.x >= counters[1]) return;
  const int t = (int)split_list[blockIdx.x];
  const uint32_t nch = tile_chunks[t];
  const uint32_t slot = tile_slot[t];
  const int T = g.T;
  int k, oy, ox;
  tile_origin(g, t, k, oy, ox);
  cplx<R>* dst = planes + ((size_t)k * g.nv + oy) * g.nu + ox;
  const R cn = (R)g.cnorm;
  const size_t tt = (size_t)T * T;
  for (int i = threadIdx.x; i < T * T; i += blockDim.x) {
    const cplx<R>* src = partials + (size_t)slot * tt + i;
    cplx<R> acc = {(R)0, (R)0};
    uint32_t c = 0;
    for (; c + 4 <= nch; c += 4) {
      const cplx<R> a0 = src[(c + 0) * tt], a1 = src[(c + 1) * tt];
      const cplx<R> a2 = src[(c + 2) * tt], a3 = src[(c + 3) * tt];
      acc = cadd(acc, a0);
      acc = cadd(acc, a1);
      acc = cadd(acc, a2);
      acc = cadd(acc, a3);
    }
    for (; c < nch; ++c) acc = cadd(acc, src[c * tt]);
    const int li = i % T, lj = i / T;
    cplx<R> v = {cn * acc.re, cn * acc.im};
    cplx<R>* p = dst + (size_t)lj * g.nu + li;
    if (accumulate) v = cadd(*p, v);
    *p = v;
  }
}

template <typename R, int K>
__global__ __launch_bounds__(256) void k_degrid_tiles(
    Geo g, const uint32_t* __restrict__ offsets,
    uint32_t* __restrict__ counters, const uint2* __restrict__ extra,
    const uint32_t* __restrict__ busy,
    const cplx<R>* __restrict__ planes, const uint32_t* __restrict__ rec_cell,
    const cplx<R>* __restrict__ rec_dxy, const cplx<R>* __restrict__ rec_val,
    const uint32_t* __restrict__ rec_idx, uint32_t chunk,
    cplx<R>* __restrict__ vis_out) {
  constexpr int H = (K - 1) / 2;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t s_item;
  cplx<R>* s_q = reinterpret_cast<cplx<R>*>(smem);
  const int T = g.T;
  const int W = T + 2 * H;
  const R cn = (R)g.cnorm;
  Item it;
  while (next_item(counters, counters, extra, busy, false, &s_item, it)) {
    const int t = it.tile;
    const uint32_t c = it.chunk;
    int k, oy, ox;
    tile_origin(g, t, k, oy, ox);
    const uint32_t r0 = offsets[(uint32_t)t * kRegions];
    const uint32_t r1 = offsets[(uint32_t)t * kRegions + kRegions];
    const uint32_t start = r0 + c * chunk;
    if (start >= r1) continue;
    const uint32_t end = r1 - start > chunk ? start + chunk : r1;
    const cplx<R>* src = planes + (size_t)k * g.nv * g.nu;
    for (int i = threadIdx.x; i < W * W; i += blockDim.x) {
      const int lr = i / W, lc = i - lr * W;
      const int gr = oy - H + lr, gc = ox - H + lc;
      cplx<R> v = {(R)0, (R)0};
      if ((unsigned)gr < (unsigned)g.nv && (unsigned)gc < (unsigned)g.nu)
        v = src[(size_t)stack_row(g, gr) * g.nu + gc];
      s_q[i] = v;
    }
    lds_barrier();
    for (uint32_t r = start + threadIdx.x; r < end; r += blockDim.x) {
      const uint32_t cc = rec_cell[r];
      const cplx<R> dxy = rec_dxy[r];
      const int li = cell_i(cc) - ox + H;
      const int lj = cell_j(cc) - oy + H;
      R gx[K], gy[K];
#pragma unroll
      for (int a = 0; a < K; ++a) {
        gx[a] = gauss1(g, (R)(a - H) - dxy.re);
        gy[a] = gauss1(g, (R)(a - H) - dxy.im);
      }
      cplx<R> acc = {(R)0, (R)0};
#pragma unroll
      for (int b = 0; b < K; ++b) {
        const int row = lj + b - H;
        if ((unsigned)row >= (unsigned)W) continue;
        cplx<R> racc = {(R)0, (R)0};
#pragma unroll
        for (int a = 0; a < K; ++a) {
          const int col = li + a - H;
          if ((unsigned)col < (unsigned)W) {
            const cplx<R> q = s_q[row * W + col];
            racc.re += gx[a] * q.re;
            racc.im += gx[a] * q.im;
          }
        }
        acc.re += gy[b] * racc.re;
        acc.im += gy[b] * racc.im;
      }
      const R wt = rec_val[r].re;
      vis_out[rec_idx[r]] = cplx<R>{cn * wt * acc.re, cn * wt * acc.im};
    }
  }
}

// Persistent workgroups: as many as fit on the device at once (bounded by
// LDS), never more than there are items.
uint32_t persistent_groups(size_t lds_bytes, int cus, uint32_t max_items) {
  const size_t lds_cu = 160 * 1024;
  size_t per_cu = lds_cu / (lds_bytes + 1024);
  if (per_cu < 1) per_cu = 1;
  if (per_cu > 8) per_cu = 8;
  uint64_t n = (uint64_t)per_cu * (uint64_t)(cus > 0 ? cus : 256);
  if (n > max_items) n = max_items;
  return (uint32_t)(n > 0 ? n : 1);
}

template <typename R, int K>
void grid_k(const GridJob<R>& j, uint32_t max_items, int cus,
            hipStream_t st) {
  const size_t lds = (size_t)2 * j.g.T * j.pitch * sizeof(double);
  hipLaunchKernelGGL((k_grid_tiles<R, K>),
                     dim3(persistent_groups(lds, cus, max_items)),
                     dim3(kGridThreads), lds, st, j);
}

template <typename R, int K>
void grid_batch_k(const GridJob<R>* jobs, int njobs, size_t lds,
                  uint32_t* queue, uint32_t max_items, int cus,
                  hipStream_t st) {
  hipLaunchKernelGGL((k_grid_batch<R, K>),
                     dim3(persistent_groups(lds, cus, max_items)),
                     dim3(kGridThreads), lds, st, jobs, njobs, queue,
                     (uint32_t)(lds / sizeof(double)));
}

template <typename R, int K>
void degrid_k(const Geo& g, const uint32_t* offsets, uint32_t* counters,
              const uint2* extra, const uint32_t* busy, const void* planes,
              const uint32_t* rec_cell, const void* rec_dxy,
              const void* rec_val, const uint32_t* rec_idx, uint32_t chunk,
              void* vis_out, uint32_t max_items, int cus, hipStream_t st) {
  const int W = g.T + (K - 1);
  const size_t lds = (size_t)W * W * sizeof(cplx<R>);
  hipLaunchKernelGGL((k_degrid_tiles<R, K>),
                     dim3(persistent_groups(lds, cus, max_items)), dim3(256),
                     lds, st, g, offsets, counters, extra, busy,
                     (const cplx<R>*)planes, rec_cell,
                     (const cplx<R>*)rec_dxy, (const cplx<R>*)rec_val,
                     rec_idx, chunk, (cplx<R>*)vis_out);
}

}  // namespace

int grid_lds_pitch(int T, int K) {
  // Row pitch in FP64 accumulators: T + K is odd, so the K rows of one
  // footprint start 2 (T + K) words apart and fall in distinct banks.
  return T + K;
}

#define WS_K_SWITCH(KVAR, CALL)                                           \
  switch (KVAR) {                                                         \
    case 1: { constexpr int KK = 1; CALL; } break;                        \
    case 3: { constexpr int KK = 3; CALL; } break;                        \
    case 5: { constexpr int KK = 5; CALL; } break;                        \
    case 7: { constexpr int KK = 7; CALL; } break;                        \
    case 9: { constexpr int KK = 9; CALL; } break;                        \
    case 11: { constexpr int KK = 11; CALL; } break;                      \
    case 13: { constexpr int KK = 13; CALL; } break;                      \
    case 15: { constexpr int KK = 15; CALL; } break;                      \
    default: break;                                                       \
  }

template <typename R>
void launch_grid_tiles(const GridJob<R>& j, uint32_t max_items, int cus,
                       hipStream_t st) {
  WS_K_SWITCH(j.g.K, (grid_k<R, KK>(j, max_items, cus, st)));
}

template <typename R>
void launch_grid_batch(const GridJob<R>* jobs, int njobs, int K, size_t lds,
                       uint32_t* queue, uint32_t max_items, int cus,
                       hipStream_t st) {
  WS_K_SWITCH(K, (grid_batch_k<R, KK>(jobs, njobs, lds, queue, max_items,
                                      cus, st)));
}

template <typename R>
void launch_grid_merge(const Geo& g, const uint32_t* counters,
                       const uint32_t* split_list, const uint32_t* tile_chunks,
                       const uint32_t* tile_slot, const void* partials,
                       void* planes, int accumulate, uint32_t max_split,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_grid_merge<R>, dim3(max_split), dim3(1024), 0, st, g,
                     counters, split_list, tile_chunks, tile_slot,
                     (const cplx<R>*)partials, (cplx<R>*)planes, accumulate);
}

template <typename R>
void launch_degrid_tiles(const Geo& g, const uint32_t* offsets,
                         uint32_t* counters, const uint2* extra,
                         const uint32_t* busy, const void* planes,
                         const uint32_t* rec_cell,
                         const void* rec_dxy, const void* rec_val,
                         const uint32_t* rec_idx, uint32_t chunk,
                         void* vis_out, uint32_t max_items, int cus,
                         hipStream_t st) {
  WS_K_SWITCH(g.K, (degrid_k<R, KK>(g, offsets, counters, extra, busy,
                                    planes,
                                    rec_cell, rec_dxy, rec_val, rec_idx,
                                    chunk, vis_out, max_items, cus, st)));
}

#undef WS_K_SWITCH

size_t degrid_lds_bytes(int T, int K, int elem_bytes) {
  const int W = T + K - 1;
  return (size_t)W * W * elem_bytes;
}

#define WS_INST(R)                                                          \
  template void launch_grid_tiles<R>(const GridJob<R>&, uint32_t, int,     \
                                     hipStream_t);                         \
  template void launch_grid_batch<R>(const GridJob<R>*, int, int, size_t,  \
                                     uint32_t*, uint32_t, int,             \
                                     hipStream_t);                         \
  template void launch_grid_merge<R>(const Geo&, const uint32_t*,          \
                                     const uint32_t*, const uint32_t*,     \
                                     const uint32_t*, const void*, void*,  \
                                     int, uint32_t, hipStream_t);          \
  template void launch_degrid_tiles<R>(                                    \
      const Geo&, const uint32_t*, uint32_t*, const uint2*,                \
      const uint32_t*, const void*,                                        \
      const uint32_t*, const void*, const void*, const uint32_t*,          \
      uint32_t, void*, uint32_t, int, hipStream_t);
WS_INST(float)
WS_INST(double)
#undef WS_INST

}  // namespace ws
