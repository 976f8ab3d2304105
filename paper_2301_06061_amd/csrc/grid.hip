// Gridding (Eq. 3) and degridding (its adjoint) over binned records.
//
// Gridding: persistent workgroups (as many as fit on the device) take work
// items (tile, chunk) from a queue in device memory.  A tile lives in LDS
// as separate real and imaginary rows of FP64 accumulators on both
// precision paths: on this part LDS FP64 atomic adds run about 20x faster
// than FP32 ones (measured, 6.6 vs 0.33 lanes per clock per CU), so the
// FP32 path computes its taps in FP32 and sums them in FP64 before rounding
// the finished tile to FP32.  A wavefront takes one visibility at a time
// and its lanes cover the K x K kernel taps, so the adds of one LDS
// instruction hit distinct cells (no same-address serialisation, even in a
// dense core where many visibilities share a cell); the LDS row pitch is
// T + K (odd), so they also fall in distinct banks.
// A tile is written to HBM once, zeros included, with 16-byte row stores;
// tiles with more records than one chunk are split over several items
// whose partial tiles a merge kernel sums in a fixed order.  Records of a
// neighbouring tile whose footprint crosses the tile edge are read from
// that tile's edge-strip bins, so no record is stored twice.  The queue
// hands out the extra chunks of split (hot) tiles first.
//
// Degridding: persistent workgroups take (tile, chunk) items; each loads
// the transformed plane's tile plus an h-cell halo into LDS once, and each
// lane evaluates one visibility's K x K weighted sum from LDS.
#include "ws_kernels.h"

namespace ws {

namespace {

constexpr int kGridThreads = 512;

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

// Work items of one plan, in queue order: the further chunks of split
// (hot) tiles, then the first chunk of every tile that has records, then -
// when idle tiles must be written - groups of kZeroGroup tiles without
// records, which only get zeros.
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

// Pop the next item of a plan's own queue (counters[3]).  Contains the
// barriers that order LDS reuse between items.
__device__ __forceinline__ bool next_item(const uint32_t* counters_ro,
                                          uint32_t* counters,
                                          const uint2* extra,
                                          const uint32_t* busy, bool with_zero,
                                          uint32_t* s_item, Item& it) {
  __syncthreads();
  if (threadIdx.x == 0) *s_item = atomicAdd(&counters[3], 1u);
  __syncthreads();
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
// path precision, 16 bytes per store.
template <typename R>
__device__ __forceinline__ void store_tile(const double* s_re,
                                           const double* s_im, int pitch,
                                           int T, double scale, cplx<R>* dst,
                                           size_t dst_pitch,
                                           bool accumulate) {
  constexpr int V = 16 / sizeof(cplx<R>);  // complex values per store
  const int per_row = T / V;
  for (int i = threadIdx.x; i < T * per_row; i += blockDim.x) {
    const int lj = i / per_row, li = (i - lj * per_row) * V;
    cplx<R> v[V];
#pragma unroll
    for (int e = 0; e < V; ++e)
      v[e] = {(R)(scale * s_re[lj * pitch + li + e]),
              (R)(scale * s_im[lj * pitch + li + e])};
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

// Gridding of one item (tile t, chunk c) of one job; called by all threads
// of the workgroup.  Each wavefront loads 64 records with one coalesced
// load per field, then takes them one at a time: its lanes cover the K*K
// taps of the visibility (in ceil(K*K/64) rounds), so the LDS adds of one
// instruction hit K*K distinct cells - no two lanes ever add to the same
// accumulator at once, even where many visibilities share a cell.
template <typename R, int K>
__device__ __forceinline__ void grid_item(const GridJob<R>& j, const Item& it,
                                          double* s_re, double* s_im) {
  constexpr int H = (K - 1) / 2;
  constexpr int KK = K * K;
  constexpr int ROUNDS = (KK + 63) / 64;
  const Geo& g = j.g;
  const int T = g.T;
  if (it.zero) {
    const uint32_t nidle = j.counters[5];
    for (uint32_t z = it.chunk * kZeroGroup;
         z < nidle && z < (it.chunk + 1) * kZeroGroup; ++z) {
      int k, oy, ox;
      tile_origin(g, (int)j.idle[z], k, oy, ox);
      zero_tile(T, j.planes + ((size_t)k * g.nv + oy) * g.nu + ox,
                (size_t)g.nu);
    }
    return;
  }
  const int t = it.tile;
  const uint32_t c = it.chunk;
  const int pitch = j.pitch;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
  const uint32_t nch = j.tile_chunks[t];
  int k, oy, ox;
  tile_origin(g, t, k, oy, ox);
  cplx<R>* dst = j.planes + ((size_t)k * g.nv + oy) * g.nu + ox;
  // Key ranges of the records that reach this tile; all offsets are loaded
  // up front so that their latencies overlap.
  uint32_t lo[10], hi[10], s0[10], len[10];
  const int ns = tile_segments(g, t, lo, hi);
  uint32_t work = 0;
#pragma unroll
  for (int s = 0; s < 10; ++s) {
    s0[s] = 0;
    len[s] = 0;
    if (s < ns) {
      s0[s] = j.offsets[lo[s]];
      len[s] = j.offsets[hi[s]] - s0[s];
    }
    work += len[s];
  }
  if (work == 0) {
    // Empty tile: the first gridding call writes its zeros; later calls
    // have nothing to add.
    if (!j.accumulate) zero_tile(T, dst, (size_t)g.nu);
    return;
  }
  for (int i = threadIdx.x; i < T * pitch; i += blockDim.x) {
    s_re[i] = 0.0;
    s_im[i] = 0.0;
  }
  int ta[ROUNDS], tb[ROUNDS];
#pragma unroll
  for (int q = 0; q < ROUNDS; ++q) {
    const int tt = lane + 64 * q;
    ta[q] = tt % K - H;
    tb[q] = tt / K - H;
  }
  __syncthreads();
  // This item's records: [c * chunk, (c + 1) * chunk) of the concatenated
  // segments; a tile gridded by a single item takes all of them.
  uint32_t skip = c * j.chunk;
  uint32_t left = nch == 1 ? work : j.chunk;
  for (int s = 0; s < ns && left > 0; ++s) {
    if (skip >= len[s]) {
      skip -= len[s];
      continue;
    }
    const uint32_t start = s0[s] + skip;
    const uint32_t n = (len[s] - skip) < left ? (len[s] - skip) : left;
    skip = 0;
    left -= n;
    for (uint32_t b0 = (uint32_t)wave * 64; b0 < n;
         b0 += (uint32_t)nwaves * 64) {
      const uint32_t my = b0 + lane;
      uint32_t cell = 0;
      cplx<R> dxy = {(R)0, (R)0}, val = {(R)0, (R)0};
      if (my < n) {
        cell = j.rec_cell[start + my];
        dxy = j.rec_dxy[start + my];
        val = j.rec_val[start + my];
      }
      const int cnt = (n - b0) < 64u ? (int)(n - b0) : 64;
      for (int r = 0; r < cnt; ++r) {
        const uint32_t cc = bcast_u(cell, r);
        const R dx = bcast(dxy.re, r), dy = bcast(dxy.im, r);
        const R vr = bcast(val.re, r), vi = bcast(val.im, r);
        const int ci = cell_i(cc) - ox, cj = cell_j(cc) - oy;
#pragma unroll
        for (int q = 0; q < ROUNDS; ++q) {
          if (KK % 64 == 0 || lane + 64 * q < KK) {
            const int li = ci + ta[q], lj = cj + tb[q];
            if ((unsigned)li < (unsigned)T && (unsigned)lj < (unsigned)T) {
              const R ex = (R)ta[q] - dx, ey = (R)tb[q] - dy;
              const R w = gauss2(g, ex * ex + ey * ey);
              atomicAdd(s_re + lj * pitch + li, (double)(w * vr));
              atomicAdd(s_im + lj * pitch + li, (double)(w * vi));
            }
          }
        }
      }
    }
  }
  __syncthreads();
  if (nch == 1) {
    store_tile(s_re, s_im, pitch, T, g.cnorm, dst, (size_t)g.nu,
               j.accumulate != 0);
  } else {
    cplx<R>* part = j.partials + (size_t)(j.tile_slot[t] + c) * T * T;
    store_tile(s_re, s_im, pitch, T, 1.0, part, (size_t)T, false);
  }
}

template <typename R, int K>
__global__ __launch_bounds__(kGridThreads) void k_grid_tiles(GridJob<R> j) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t s_item;
  double* s_re = reinterpret_cast<double*>(smem);
  double* s_im = s_re + j.g.T * j.pitch;
  Item it;
  while (next_item(j.counters, j.counters, j.extra, j.busy, !j.accumulate,
                   &s_item, it))
    grid_item<R, K>(j, it, s_re, s_im);
}

// Batched gridding: one persistent launch drains a single queue holding the
// work items of every job (plan), job after job; the LDS tile is sized for
// the largest tile of the batch.
template <typename R, int K>
__global__ __launch_bounds__(kGridThreads) void k_grid_batch(
    const GridJob<R>* __restrict__ jobs, int njobs,
    uint32_t* __restrict__ queue) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t s_item;
  __shared__ uint32_t s_base[kMaxBatch + 1];
  double* s_re = reinterpret_cast<double*>(smem);
  if (threadIdx.x == 0) {
    uint32_t b = 0;
    for (int p = 0; p < njobs; ++p) {
      s_base[p] = b;
      b += item_total(jobs[p].counters, !jobs[p].accumulate);
    }
    s_base[njobs] = b;
  }
  while (true) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(queue, 1u);
    __syncthreads();
    const uint32_t item = s_item;
    if (item >= s_base[njobs]) break;
    int p = 0;
    while (item >= s_base[p + 1]) ++p;
    const GridJob<R> j = jobs[p];
    const Item it = resolve_item(item - s_base[p], j.counters, j.extra, j.busy);
    grid_item<R, K>(j, it, s_re, s_re + j.g.T * j.pitch);
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
    __syncthreads();
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
                     dim3(kGridThreads), lds, st, jobs, njobs, queue);
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
