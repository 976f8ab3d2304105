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
// Degridding: one workgroup per (tile, chunk) item (the hardware overlaps
// the latencies of the workgroups resident on a CU); each loads the
// transformed plane's tile plus an h-cell halo into LDS in one round trip,
// and each lane evaluates one visibility's K x K weighted sum from LDS.
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

// One-dimensional kernel factor phi(d) at offset d (cells) from the
// visibility, for |d| <= K/2 (the taps of the K x K footprint).
//   Gaussian: exp(-d^2 / (2 sigma^2)); FP32 takes the hardware base-2
//     exponential (v_exp_f32) of a pre-scaled argument, never near its
//     denormal range (the farthest tap of the widest kernel is >= 2^-30).
//   ES: exp(beta (sqrt(1 - z^2) - 1)) = exp(-beta z^2 / (1 + sqrt(1 - z^2))),
//     the second form free of cancellation near the centre; 1 - z^2 is
//     clamped at 0 (rounding can take |z| a hair past 1 at the edge tap).
template <int KT>
__device__ __forceinline__ float kern1(const Geo& g, float d) {
  if constexpr (KT == kKernelES) {
    const float z = d * g.es_zs_f;
    const float z2 = z * z;
    const float t = 1.0f - z2 > 0.0f ? 1.0f - z2 : 0.0f;
    return __builtin_amdgcn_exp2f(-g.es_beta2 * z2 / (1.0f + __builtin_sqrtf(t)));
  } else {
    return __builtin_amdgcn_exp2f(-g.kappa * (d * d));
  }
}
template <int KT>
__device__ __forceinline__ double kern1(const Geo& g, double d) {
  if constexpr (KT == kKernelES) {
    const double z = d * g.es_zs;
    const double z2 = z * z;
    const double t = 1.0 - z2 > 0.0 ? 1.0 - z2 : 0.0;
    return exp(-g.es_beta * z2 / (1.0 + sqrt(t)));
  } else {
    return exp(-g.inv2s2 * (d * d));
  }
}

struct Item {
  int tile;
  uint32_t chunk;  // chunk of the tile
};

// Work items of one plan, in queue order: the further chunks of split
// (hot) tiles, then the first chunk of every tile that has records.
__device__ __forceinline__ uint32_t item_total(const uint32_t* counters) {
  return counters[2] + counters[4];
}

__device__ __forceinline__ Item resolve_item(uint32_t item,
                                             const uint32_t* counters,
                                             const uint2* extra,
                                             const uint32_t* busy) {
  const uint32_t nextra = counters[2];
  Item it;
  if (item < nextra) {
    const uint2 tc = extra[item];
    it.tile = (int)tc.x;
    it.chunk = tc.y;
  } else {
    it.tile = (int)busy[item - nextra];
    it.chunk = 0;
  }
  return it;
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

// Store (or add) a T x T tile of LDS accumulators (type A), held as
// separate real and imaginary rows, into a row-major complex destination of
// the path precision, 16 bytes per store; the LDS cells read are cleared.
// BLOCKED: the destination is a slot of the busy-tile store instead
// (tile_store_at; dst_pitch unused).  Consecutive threads take
// consecutive cells of a row either way, which keeps the LDS reads free
// of bank conflicts; in the store, the two rows a wavefront covers are
// adjacent in every 64-byte column sub-block.
template <typename R, typename A, bool BLOCKED = false>
__device__ __forceinline__ void store_tile_clear(A* s_re, A* s_im,
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
      s_re[a] = (A)0;
      s_im[a] = (A)0;
    }
    static_assert(!BLOCKED || (64 / sizeof(cplx<R>)) % V == 0,
                  "a store stays inside one column sub-block");
    cplx<R>* p = BLOCKED ? dst + tile_store_at<R>(T, lj, li)
                         : dst + (size_t)lj * dst_pitch + li;
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

__device__ __forceinline__ uint32_t uniform(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

template <typename R>
struct RecBatch {
  uint32_t cell;
  cplx<R> dxy, val;
};

// A work item resolved for gridding (uniform across the workgroup except
// `first`).  The records of a tile are the concatenation of its key
// ranges; position f of that list is record f + off0 + the sum of step[s]
// over the ranges s >= 1 with cum[s] <= f.  The item covers positions
// [f0, f1).  `first` is this thread's share of the item's first batch of
// records, loaded while the previous item is still being written out
// (loads and stores complete in order, so a load issued after a tile's
// stores would wait for them).
template <typename R>
struct GridItem {
  int valid;
  int tile;
  uint32_t nch;    // items the tile is split into
  uint32_t chunk;  // which of them; a tile of one chunk: its busy index
  uint32_t f0, f1;
  uint32_t off0;
  uint32_t cum[kSegments];
  uint32_t step[kSegments];
  RecBatch<R> first;
};

// Record index of list position f of item x (a sum of selects, so that
// the per-range values stay in registers).
template <typename R>
__device__ __forceinline__ uint32_t record_at(const GridItem<R>& x,
                                              uint32_t f) {
  uint32_t r = f + x.off0;
#pragma unroll
  for (int s = 1; s < kSegments; ++s) r += f >= x.cum[s] ? x.step[s] : 0u;
  return r;
}

// Loads list position f of the item for a share that ends at `end`;
// positions past the end re-read the share's last record (so the loads
// need no branch) and give a zero value.
template <typename R>
__device__ __forceinline__ RecBatch<R> load_batch(const GridJob<R>& j,
                                                  const GridItem<R>& x,
                                                  uint32_t f, uint32_t end) {
  const bool in = f < end;
  const uint32_t r = record_at(x, in ? f : end - 1);
  const Record<R> q = j.rec[r];
  RecBatch<R> b;
  b.cell = q.cell;
  b.dxy = {q.dx, q.dy};
  b.val = {in ? q.vr : (R)0, in ? q.vi : (R)0};
  return b;
}

// Share of wavefront w (of nw) in the item's list positions [f0, f1):
// consecutive runs of equal length, so that every wavefront has work even
// in a tile with few records.
__device__ __forceinline__ void wave_share(uint32_t f0, uint32_t f1, int w,
                                           int nw, uint32_t& b, uint32_t& e) {
  const uint32_t q = (f1 - f0 + (uint32_t)nw - 1) / (uint32_t)nw;
  b = f0 + (uint32_t)w * q;
  e = min(b + q, f1);
}

// Work item descriptors: everything the gridder needs to start an item,
// written by k_item_desc after the tile work pass, so that the gridder
// starts an item with one load instead of a chain of dependent loads (queue
// entry -> tile -> its key ranges).  Words: tile, chunks of the tile, chunk,
// f0, f1, off0, cum[1 .. kSegments-1], step[1 .. kSegments-1].  A tile of
// one chunk (chunk 0, never an extra item) has its index in the busy list
// in the chunk word instead: its slot in the busy-tile store.
static_assert(6 + 2 * (kSegments - 1) == kDescWords, "descriptor layout");

__global__ __launch_bounds__(256) void k_item_desc(
    Geo g, const uint32_t* __restrict__ offsets,
    const uint32_t* __restrict__ counters, const uint2* __restrict__ extra,
    const uint32_t* __restrict__ busy,
    const uint32_t* __restrict__ tile_chunks, uint32_t chunk,
    uint32_t* __restrict__ desc, uint32_t max_items) {
  const uint32_t n = blockIdx.x * 256u + threadIdx.x;
  if (n >= max_items) return;
  const uint32_t nextra = counters[2];
  if (n >= nextra + counters[4]) return;
  const bool is_extra = n < nextra;
  const uint32_t tile = is_extra ? extra[n].x : busy[n - nextra];
  const uint32_t ch = is_extra ? extra[n].y : 0u;
  const uint32_t nch = tile_chunks[tile];
  uint32_t lo[kSegments], hi[kSegments];
  tile_segments(g, (int)tile, lo, hi);
  uint32_t w[kDescWords];
  uint32_t cum = 0, prev = 0;
#pragma unroll
  for (int s = 0; s < kSegments; ++s) {
    const uint32_t as = offsets[lo[s]], bs = offsets[hi[s]];
    const uint32_t off = as - cum;
    if (s == 0) {
      w[5] = off;
    } else {
      w[5 + s] = cum;
      w[5 + kSegments - 1 + s] = off - prev;
    }
    prev = off;
    cum += bs - as;
  }
  const uint32_t f0 = ch * chunk;
  w[0] = tile;
  w[1] = nch;
  w[2] = nch == 1 ? n - nextra : ch;
  w[3] = f0;
  w[4] = nch == 1 ? cum : min(cum, f0 + chunk);
  uint4* d = reinterpret_cast<uint4*>(desc + (size_t)n * kDescWords);
#pragma unroll
  for (int q = 0; q < kDescWords / 4; ++q)
    d[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
}

// A descriptor as loaded (uniform values; left in whatever registers the
// loads produce until the item starts, so nothing waits for them early).
struct DescRegs {
  uint32_t w[kDescWords];
};

__device__ __forceinline__ DescRegs load_desc(const uint32_t* __restrict__ desc,
                                              uint32_t n, bool valid) {
  DescRegs d;
  const uint32_t* p = desc + (size_t)(valid ? n : 0u) * kDescWords;
#pragma unroll
  for (int i = 0; i < kDescWords; ++i) d.w[i] = p[i];
  return d;
}

// The item of a loaded descriptor, with this thread's share of its first
// batch of records requested.
template <typename R>
__device__ __forceinline__ GridItem<R> item_from(const GridJob<R>& j,
                                                 const DescRegs& d,
                                                 bool valid) {
  GridItem<R> x;
  x.valid = valid;
  x.tile = (int)uniform(valid ? d.w[0] : 0u);
  x.nch = uniform(valid ? d.w[1] : 1u);
  x.chunk = uniform(valid ? d.w[2] : 0u);
  x.f0 = uniform(valid ? d.w[3] : 0u);
  x.f1 = uniform(valid ? d.w[4] : 0u);
  x.off0 = uniform(valid ? d.w[5] : 0u);
  x.cum[0] = x.step[0] = 0;
#pragma unroll
  for (int s = 1; s < kSegments; ++s) {
    x.cum[s] = uniform(valid ? d.w[5 + s] : 0u);
    x.step[s] = uniform(valid ? d.w[5 + kSegments - 1 + s] : 0u);
  }
  x.first.cell = 0;
  x.first.dxy = x.first.val = {(R)0, (R)0};
  if (x.f1 > x.f0) {
    uint32_t b, e;
    wave_share(x.f0, x.f1, threadIdx.x >> 6, blockDim.x >> 6, b, e);
    x.first = load_batch(j, x, b + (threadIdx.x & 63), e);
  }
  return x;
}

// Lanes of the accumulation: lane = slot * K + row, slot < RPW.  A group
// of RPW records is added at once, each by K lanes, one kernel row per
// lane (K = 7: 9 records on 63 lanes); a batch of the wavefront's record
// loads (one record per lane) holds NG groups.
template <int K>
struct RowLanes {
  static constexpr int RPW = 64 / K;   // records per group
  static constexpr int NG = 64 / RPW;  // groups per batch
  static constexpr int BS = RPW * NG;  // records per batch (<= 64)
};

// Kernel weights of one row of taps, phi(a - H - dx) for a = 0 .. K-1.
// FP32, and the FP64 ES kernel: one kernel evaluation per tap.  FP64
// Gaussian: the ratio of neighbouring taps, q(a) = w(a+1) / w(a), itself
// changes by the constant factor d = exp(-1 / sigma^2), so a row costs two
// exps and two products a tap (relative rounding a few ulps of FP64).  The
// recurrence starts at the far-left tap, whose weight underflows (and the
// first ratio overflows) once (h + 1/2)^2 / (2 sigma^2) nears the FP64
// exponent range; such narrow kernels (`direct`, a uniform flag) take one
// exp per tap instead.
template <typename R, int K, int KT>
struct RowWeights {
  const Geo& g;
  R dx;
  __device__ __forceinline__ RowWeights(const Geo& g_, R dx_, double)
      : g(g_), dx(dx_) {}
  __device__ __forceinline__ R at(int a) {
    return kern1<KT>(g, (R)(a - (K - 1) / 2) - dx);
  }
};
template <int K>
struct RowWeights<double, K, kKernelGauss> {
  double w, q, d, dx, inv2s2;
  bool direct;
  __device__ __forceinline__ RowWeights(const Geo& g, double dx_, double d_) {
    const double e0 = (double)(-(K - 1) / 2) - dx_;
    // (h + 1)^2 / (2 sigma^2) bounds the exponents of w and q below.
    direct = g.inv2s2 * (double)(((K + 1) / 2) * ((K + 1) / 2)) > 500.0;
    w = exp(-g.inv2s2 * (e0 * e0));
    q = direct ? 0.0 : exp(-g.inv2s2 * (2.0 * e0 + 1.0));
    d = d_;
    dx = dx_;
    inv2s2 = g.inv2s2;
  }
  __device__ __forceinline__ double at(int a) {
    if (direct) {
      const double ex = (double)(a - (K - 1) / 2) - dx;
      return exp(-inv2s2 * (ex * ex));
    }
    const double v = w;
    w *= q;
    q *= d;
    return v;
  }
};

// Adds kernel row `row` of one record to the LDS tile (taps outside the
// tile belong to a neighbouring tile and are skipped).
template <typename R, int K, int KT>
__device__ __forceinline__ void add_row(const Geo& g, uint32_t cc, R dx, R dy,
                                        R vr, R vi, int row, int ox, int oy,
                                        int T, int pitch, double d,
                                        GridAcc<R>* s_re, GridAcc<R>* s_im) {
  constexpr int H = (K - 1) / 2;
  const int ci = cell_i(cc) - ox - H;  // tile column of tap 0
  const int lj = cell_j(cc) - oy + row - H;
  if ((unsigned)lj >= (unsigned)T) return;
  const R ey = (R)(row - H) - dy;
  const R gy = kern1<KT>(g, ey);
  const R wr = gy * vr, wi = gy * vi;
  GridAcc<R>* pre = s_re + lj * pitch + ci;
  GridAcc<R>* pim = s_im + lj * pitch + ci;
  RowWeights<R, K, KT> rw(g, dx, d);
#pragma unroll
  for (int a = 0; a < K; ++a) {
    const R gx = rw.at(a);
    if ((unsigned)(ci + a) < (unsigned)T) {
      atomicAdd(pre + a, (GridAcc<R>)(gx * wr));
      atomicAdd(pim + a, (GridAcc<R>)(gx * wi));
    }
  }
}

template <typename R>
__device__ __forceinline__ R lane_value(R x, int src) {
  return __shfl(x, src, 64);
}
__device__ __forceinline__ uint32_t lane_value_u(uint32_t x, int src) {
  return (uint32_t)__shfl((int)x, src, 64);
}

// Accumulates the item's records into the LDS tile.  Each wavefront takes
// an equal run of the item's list positions, BS at a time (one record per
// lane), with the next BS in flight while the current ones are added a
// group of RPW records at a time (lane values moved by lane permutes).
template <typename R, int K, int KT>
__device__ __forceinline__ void accumulate_item(const GridJob<R>& j,
                                                const GridItem<R>& x,
                                                GridAcc<R>* s_re,
                                                GridAcc<R>* s_im) {
  using RL = RowLanes<K>;
  const int T = j.g.T;
  const int pitch = j.pitch;
  const int lane = threadIdx.x & 63;
  const int slot = lane / K;
  const int row = lane - slot * K;
  const bool act = slot < RL::RPW;
  const int src0 = act ? slot : 0;
  // FP64 weights: the factor between neighbouring tap ratios.
  const double d = sizeof(R) == 8 ? exp(-2.0 * j.g.inv2s2) : 0.0;
  int k, oy, ox;
  tile_origin(j.g, x.tile, k, oy, ox);
  uint32_t b0, e;
  wave_share(x.f0, x.f1, threadIdx.x >> 6, blockDim.x >> 6, b0, e);
  RecBatch<R> cur = x.first;
  while (b0 < e) {
    const uint32_t b1 = b0 + (uint32_t)RL::BS;
    const RecBatch<R> nxt = load_batch(j, x, b1 + lane, e);
    const int cnt = (e - b0) < (uint32_t)RL::BS ? (int)(e - b0) : RL::BS;
#pragma unroll
    for (int gq = 0; gq < RL::NG; ++gq) {
      if (gq * RL::RPW >= cnt) break;
      const int src = gq * RL::RPW + src0;
      const uint32_t cc = lane_value_u(cur.cell, src);
      const R dx = lane_value(cur.dxy.re, src), dy = lane_value(cur.dxy.im, src);
      const R vr = lane_value(cur.val.re, src), vi = lane_value(cur.val.im, src);
      if (act && src < cnt)
        add_row<R, K, KT>(j.g, cc, dx, dy, vr, vi, row, ox, oy, T, pitch, d,
                          s_re, s_im);
    }
    cur = nxt;
    b0 = b1;
  }
}

// Writes a finished item: the whole tile (scaled by the kernel norm), or
// one partial tile of a split tile.  Clears the LDS cells it reads.
// A tile whose item has no records (possible only when a later call adds
// to a tile left empty) gets zeros on a first call and nothing otherwise.
template <typename R>
__device__ __forceinline__ void store_item(const GridJob<R>& j,
                                           const GridItem<R>& x,
                                           GridAcc<R>* s_re,
                                           GridAcc<R>* s_im) {
  const int T = j.g.T;
  int k, oy, ox;
  tile_origin(j.g, x.tile, k, oy, ox);
  cplx<R>* dst = j.planes + ((size_t)k * j.g.nv + oy) * j.g.nu + ox;
  if (j.tstore != nullptr && x.nch == 1 && x.chunk < j.tcap) {
    // One-call path: the tile goes to its slot of the busy-tile store
    // (the item's busy-list index is its slot: no load of tslot here).
    cplx<R>* slot = j.tstore + (size_t)x.chunk * T * T;
    if (x.f1 <= x.f0) {
      if (!j.accumulate) zero_tile(T, slot, (size_t)T);
    } else {
      store_tile_clear<R, GridAcc<R>, true>(s_re, s_im, j.pitch, T,
                                            j.g.cnorm, slot, 0,
                                            j.accumulate != 0);
    }
  } else if (x.f1 <= x.f0) {
    if (x.nch == 1 && !j.accumulate) zero_tile(T, dst, (size_t)j.g.nu);
  } else if (x.nch == 1) {
    store_tile_clear(s_re, s_im, j.pitch, T, j.g.cnorm, dst,
                     (size_t)j.g.nu, j.accumulate != 0);
  } else {
    cplx<R>* part =
        j.partials + (size_t)(j.tile_slot[x.tile] + x.chunk) * T * T;
    store_tile_clear(s_re, s_im, j.pitch, T, 1.0, part, (size_t)T, false);
  }
}

template <typename A>
__device__ __forceinline__ void clear_lds(A* s, uint32_t words) {
  for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) s[i] = (A)0;
}

// Persistent loop over the items of a queue.  Thread 0 pops queue numbers
// into s_next; `locate(n, job)` turns number n into its job and the index
// of the item in that job (returns false past the end).  Queue numbers are
// popped two items ahead: the descriptor of the item after the current one
// is loaded while the current one accumulates, and that item's first
// records are requested before the current tile's global stores, which
// then drain while it starts.  The barriers order LDS only.
template <typename R, int K, int KT, class Locate>
__device__ __forceinline__ void item_loop(GridAcc<R>* s_lds, uint32_t* queue,
                                          uint32_t* s_next,
                                          const GridJob<R>* job0,
                                          Locate locate) {
  if (threadIdx.x == 0) {
    s_next[0] = atomicAdd(queue, 1u);
    s_next[1] = atomicAdd(queue, 1u);
  }
  lds_barrier();
  const GridJob<R>* job = job0;
  uint32_t li = 0;
  bool v = locate(uniform(s_next[0]), job, li);
  GridItem<R> x = item_from(*job, load_desc(job->desc, li, v), v);
  const GridJob<R>* jn = job0;
  bool vn = locate(uniform(s_next[1]), jn, li);
  DescRegs dn = load_desc(jn->desc, li, vn);
  while (x.valid) {
    lds_barrier();  // every thread has read s_next; LDS is clear
    if (threadIdx.x == 0) s_next[0] = atomicAdd(queue, 1u);
    const GridJob<R>& j = *job;
    GridAcc<R>* s_re = s_lds;
    GridAcc<R>* s_im = s_lds + j.g.T * j.pitch;
    if (x.f1 > x.f0) accumulate_item<R, K, KT>(j, x, s_re, s_im);
    lds_barrier();  // LDS sums complete; s_next visible
    const GridItem<R> nx = item_from(*jn, dn, vn);
    const GridJob<R>* jnn = job0;
    const bool vnn = locate(uniform(s_next[0]), jnn, li);
    dn = load_desc(jnn->desc, li, vnn);
    store_item(j, x, s_re, s_im);
    x = nx;
    job = jn;
    jn = jnn;
    vn = vnn;
  }
}

template <typename R, int K, int KT>
__global__ __launch_bounds__(kGridThreads) void k_grid_tiles(GridJob<R> j) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t s_next[2];
  GridAcc<R>* s_lds = reinterpret_cast<GridAcc<R>*>(smem);
  const uint32_t total = item_total(j.counters);
  clear_lds(s_lds, 2u * (uint32_t)(j.g.T * j.pitch));
  item_loop<R, K, KT>(s_lds, &j.counters[3], s_next, &j,
                  [&](uint32_t n, const GridJob<R>*&, uint32_t& li) {
                    li = n;
                    return n < total;
                  });
}

// Batched gridding: one persistent launch drains a single queue holding the
// work items of every job (plan), job after job; the LDS tile is sized for
// the largest tile of the batch (lds_words accumulators in all).  Jobs are
// read in place (uniform loads), never copied.
template <typename R, int K, int KT>
__global__ __launch_bounds__(kGridThreads) void k_grid_batch(
    const GridJob<R>* __restrict__ jobs, int njobs,
    uint32_t* __restrict__ queue, uint32_t lds_words) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t s_next[2];
  __shared__ uint32_t s_base[kMaxBatch + 1];
  GridAcc<R>* s_lds = reinterpret_cast<GridAcc<R>*>(smem);
  if (threadIdx.x == 0) {
    uint32_t b = 0;
    for (int p = 0; p < njobs; ++p) {
      s_base[p] = b;
      b += item_total(jobs[p].counters);
    }
    s_base[njobs] = b;
  }
  clear_lds(s_lds, lds_words);
  lds_barrier();
  item_loop<R, K, KT>(s_lds, queue, s_next, jobs,
                  [&](uint32_t n, const GridJob<R>*& jp, uint32_t& li) {
                    int p = 0;
                    const bool live = n < s_base[njobs];
                    if (live)
                      while (n >= s_base[p + 1]) ++p;
                    jp = jobs + p;
                    li = live ? n - s_base[p] : 0u;
                    return live;
                  });
}

// Zeros of the tiles without records (first gridding call of a plan):
// one workgroup per idle tile, 16-byte row stores.  Launched before the
// gridding kernel; a separate kernel keeps these HBM-bound stores at full
// rate, free of the gridder's per-item synchronisation.
template <typename R>
__device__ __forceinline__ void zero_idle_tile(const Geo& g,
                                               const uint32_t* idle,
                                               uint32_t i, cplx<R>* planes) {
  int k, oy, ox;
  tile_origin(g, (int)idle[i], k, oy, ox);
  zero_tile(g.T, planes + ((size_t)k * g.nv + oy) * g.nu + ox, (size_t)g.nu);
}

template <typename R>
__global__ __launch_bounds__(256) void k_zero_idle(
    Geo g, const uint32_t* __restrict__ counters,
    const uint32_t* __restrict__ idle, cplx<R>* __restrict__ planes) {
  if (blockIdx.x >= counters[5]) return;
  zero_idle_tile(g, idle, blockIdx.x, planes);
}

// Batched form: block b is idle entry b - base(p) of job p, where base(p)
// sums the tile counts of the jobs before p.
template <typename R>
__global__ __launch_bounds__(256) void k_zero_idle_batch(
    const GridJob<R>* __restrict__ jobs, int njobs) {
  uint32_t b = blockIdx.x;
  int p = 0;
  while (p < njobs && b >= (uint32_t)jobs[p].g.ntiles) {
    b -= (uint32_t)jobs[p].g.ntiles;
    ++p;
  }
  if (p >= njobs || !jobs[p].zero_idle || b >= jobs[p].counters[5]) return;
  zero_idle_tile(jobs[p].g, jobs[p].idle, b, jobs[p].planes);
}

template <typename R>
__global__ __launch_bounds__(1024) void k_grid_merge(
    Geo g, const uint32_t* __restrict__ counters,
    const uint32_t* __restrict__ split_list,
    const uint32_t* __restrict__ tile_chunks,
    const uint32_t* __restrict__ tile_slot,
    const cplx<R>* __restrict__ partials, cplx<R>* __restrict__ planes,
    int accumulate, cplx<R>* __restrict__ tstore,
    const uint32_t* __restrict__ tslot, uint32_t tcap) {
  // Several workgroups per split tile (blockIdx.y), each summing the
  // partials of its share of the cells in chunk order, eight loads in
  // flight per thread: the hottest tiles have tens of chunks, and the
  // chain of dependent sums per cell is what the merge waits on.
  if (blockIdx.x >= counters[1]) return;
  const int t = (int)split_list[blockIdx.x];
  const uint32_t nch = tile_chunks[t];
  const uint32_t slot = tile_slot[t];
  const int T = g.T;
  int k, oy, ox;
  tile_origin(g, t, k, oy, ox);
  const uint32_t ts = tstore != nullptr ? tslot[t] : tcap;
  const bool in_store = ts < tcap;
  cplx<R>* dst = in_store ? tstore + (size_t)ts * T * T
                          : planes + ((size_t)k * g.nv + oy) * g.nu + ox;
  const R cn = (R)g.cnorm;
  const size_t tt = (size_t)T * T;
  for (int i = blockIdx.y * blockDim.x + threadIdx.x; i < T * T;
       i += gridDim.y * blockDim.x) {
    const cplx<R>* src = partials + (size_t)slot * tt + i;
    cplx<R> acc = {(R)0, (R)0};
    uint32_t c = 0;
    for (; c + 8 <= nch; c += 8) {
      cplx<R> a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = src[(c + u) * tt];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = cadd(acc, a[u]);
    }
    for (; c < nch; ++c) acc = cadd(acc, src[c * tt]);
    const int li = i % T, lj = i / T;
    cplx<R> v = {cn * acc.re, cn * acc.im};
    cplx<R>* p = in_store ? dst + tile_store_at<R>(T, lj, li)
                          : dst + (size_t)lj * g.nu + li;
    if (accumulate) v = cadd(*p, v);
    *p = v;
  }
}

template <typename R, int K, int KT>
__global__ __launch_bounds__(256) void k_degrid_tiles(
    Geo g, const uint32_t* __restrict__ offsets,
    uint32_t* __restrict__ counters, const uint2* __restrict__ extra,
    const uint32_t* __restrict__ busy,
    const cplx<R>* __restrict__ planes, const Record<R>* __restrict__ rec,
    uint32_t chunk,
    cplx<R>* __restrict__ vis_out) {
  constexpr int H = (K - 1) / 2;
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<R>* s_q = reinterpret_cast<cplx<R>*>(smem);
  const int T = g.T;
  const int W = T + 2 * H;
  const R cn = (R)g.cnorm;
  // One workgroup per item (the hardware overlaps the latencies of the
  // workgroups resident on a CU); blocks past the item count exit.
  {
    const uint32_t item = blockIdx.x;
    if (item >= item_total(counters)) return;
    const Item it = resolve_item(item, counters, extra, busy);
    const int t = it.tile;
    const uint32_t c = it.chunk;
    int k, oy, ox;
    tile_origin(g, t, k, oy, ox);
    const uint32_t r0 = offsets[(uint32_t)t * kRegions];
    const uint32_t r1 = offsets[(uint32_t)t * kRegions + kRegions];
    const uint32_t start = r0 + c * chunk;
    if (start >= r1) return;
    const uint32_t end = r1 - start > chunk ? start + chunk : r1;
    const cplx<R>* src = planes + (size_t)k * g.nv * g.nu;
    // Tile + halo into LDS, up to kTile loads in flight per thread before
    // their LDS writes (one round trip for a 64 x 64 tile with K <= 15;
    // addresses clamped into the plane, so the loads are unconditional;
    // cells off the grid are zeroed afterwards).
    constexpr int kTile = 24;
    for (int i0 = threadIdx.x; i0 < W * W; i0 += kTile * (int)blockDim.x) {
      cplx<R> v[kTile];
#pragma unroll
      for (int u = 0; u < kTile; ++u) {
        const int i = i0 + u * (int)blockDim.x;
        const int ii = i < W * W ? i : W * W - 1;
        const int lr = ii / W, lc = ii - lr * W;
        const int gr = oy - H + lr, gc = ox - H + lc;
        const int grc = gr < 0 ? 0 : (gr >= g.nv ? g.nv - 1 : gr);
        const int gcc = gc < 0 ? 0 : (gc >= g.nu ? g.nu - 1 : gc);
        v[u] = src[(size_t)stack_row(g, grc) * g.nu + gcc];
        if (gr != grc || gc != gcc) v[u] = cplx<R>{(R)0, (R)0};
      }
#pragma unroll
      for (int u = 0; u < kTile; ++u) {
        const int i = i0 + u * (int)blockDim.x;
        if (i < W * W) s_q[i] = v[u];
      }
    }
    lds_barrier();
    // Records kRec at a time per thread, the next kRec in flight while the
    // current ones are evaluated (positions past the end re-read the last
    // record and are not written).
    constexpr int kRec = sizeof(R) == 4 ? 4 : 2;
    const uint32_t step = blockDim.x;
    auto load = [&](uint32_t r0, Record<R> (&q)[kRec]) {
#pragma unroll
      for (int u = 0; u < kRec; ++u) {
        const uint32_t r = r0 + (uint32_t)u * step;
        q[u] = rec[r < end ? r : end - 1];
      }
    };
    Record<R> cur[kRec];
    uint32_t rb = start + threadIdx.x;
    load(rb, cur);
    while (rb < end) {
      Record<R> nxt[kRec];
      const uint32_t rn = rb + (uint32_t)kRec * step;
      load(rn, nxt);
#pragma unroll
      for (int u = 0; u < kRec; ++u) {
        const Record<R>& q = cur[u];
        const int li = cell_i(q.cell) - ox + H;
        const int lj = cell_j(q.cell) - oy + H;
        R gx[K], gy[K];
#pragma unroll
        for (int a = 0; a < K; ++a) {
          gx[a] = kern1<KT>(g, (R)(a - H) - q.dx);
          gy[a] = kern1<KT>(g, (R)(a - H) - q.dy);
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
              const cplx<R> v = s_q[row * W + col];
              racc.re += gx[a] * v.re;
              racc.im += gx[a] * v.im;
            }
          }
          acc.re += gy[b] * racc.re;
          acc.im += gy[b] * racc.im;
        }
        if (rb + (uint32_t)u * step < end)
          vis_out[q.idx] = cplx<R>{cn * q.vr * acc.re, cn * q.vr * acc.im};
      }
#pragma unroll
      for (int u = 0; u < kRec; ++u) cur[u] = nxt[u];
      rb = rn;
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

template <typename R, int K, int KT>
void grid_k(const GridJob<R>& j, uint32_t max_items, int cus,
            hipStream_t st) {
  const size_t lds = grid_lds_bytes(j.g.T, K, (int)sizeof(R));
  hipLaunchKernelGGL((k_grid_tiles<R, K, KT>),
                     dim3(persistent_groups(lds, cus, max_items)),
                     dim3(kGridThreads), lds, st, j);
}

template <typename R, int K, int KT>
void grid_batch_k(const GridJob<R>* jobs, int njobs, size_t lds,
                  uint32_t* queue, uint32_t max_items, int cus,
                  hipStream_t st) {
  hipLaunchKernelGGL((k_grid_batch<R, K, KT>),
                     dim3(persistent_groups(lds, cus, max_items)),
                     dim3(kGridThreads), lds, st, jobs, njobs, queue,
                     (uint32_t)(lds / sizeof(GridAcc<R>)));
}

template <typename R, int K, int KT>
void degrid_k(const Geo& g, const uint32_t* offsets, uint32_t* counters,
              const uint2* extra, const uint32_t* busy, const void* planes,
              const void* records, uint32_t chunk,
              void* vis_out, uint32_t max_items, int cus, hipStream_t st) {
  const int W = g.T + (K - 1);
  const size_t lds = (size_t)W * W * sizeof(cplx<R>);
  hipLaunchKernelGGL((k_degrid_tiles<R, K, KT>),
                     dim3(max_items > 0 ? max_items : 1), dim3(256),
                     lds, st, g, offsets, counters, extra, busy,
                     (const cplx<R>*)planes, (const Record<R>*)records,
                     chunk, (cplx<R>*)vis_out);
}

}  // namespace

size_t grid_lds_bytes(int T, int K, int real_bytes) {
  return (size_t)2 * T * grid_lds_pitch(T, K) *
         (real_bytes == 8 ? sizeof(GridAcc<double>) : sizeof(GridAcc<float>));
}

int grid_lds_pitch(int T, int K) {
  // Row pitch in FP64 accumulators: T + K is odd, so the K rows of one
  // footprint start 2 (T + K) words apart and fall in distinct banks.
  return T + K;
}

// Dispatch on the support (KK) and the kernel type (KT), both compile-time
// specialisations of the gridding and degridding kernels.
#define WS_KT_SWITCH(KK, KTVAR, CALL)                                     \
  if ((KTVAR) == kKernelES) {                                             \
    constexpr int KT = kKernelES;                                         \
    CALL;                                                                 \
  } else {                                                                \
    constexpr int KT = kKernelGauss;                                      \
    CALL;                                                                 \
  }
#define WS_K_SWITCH(KVAR, KTVAR, CALL)                                    \
  switch (KVAR) {                                                         \
    case 1: { constexpr int KK = 1; WS_KT_SWITCH(KK, KTVAR, CALL) } break; \
    case 3: { constexpr int KK = 3; WS_KT_SWITCH(KK, KTVAR, CALL) } break; \
    case 5: { constexpr int KK = 5; WS_KT_SWITCH(KK, KTVAR, CALL) } break; \
    case 7: { constexpr int KK = 7; WS_KT_SWITCH(KK, KTVAR, CALL) } break; \
    case 9: { constexpr int KK = 9; WS_KT_SWITCH(KK, KTVAR, CALL) } break; \
    case 11: { constexpr int KK = 11; WS_KT_SWITCH(KK, KTVAR, CALL) } break; \
    case 13: { constexpr int KK = 13; WS_KT_SWITCH(KK, KTVAR, CALL) } break; \
    case 15: { constexpr int KK = 15; WS_KT_SWITCH(KK, KTVAR, CALL) } break; \
    default: break;                                                       \
  }

template <typename R>
void launch_grid_tiles(const GridJob<R>& j, uint32_t max_items, int cus,
                       hipStream_t st) {
  WS_K_SWITCH(j.g.K, j.g.kern, (grid_k<R, KK, KT>(j, max_items, cus, st)));
}

template <typename R>
void launch_grid_batch(const GridJob<R>* jobs, int njobs, int K, int kern,
                       size_t lds, uint32_t* queue, uint32_t max_items,
                       int cus, hipStream_t st) {
  WS_K_SWITCH(K, kern, (grid_batch_k<R, KK, KT>(jobs, njobs, lds, queue,
                                                max_items, cus, st)));
}

void launch_item_desc(const Geo& g, const uint32_t* offsets,
                      const uint32_t* counters, const uint2* extra,
                      const uint32_t* busy, const uint32_t* tile_chunks,
                      uint32_t chunk, uint32_t* desc, uint32_t max_items,
                      hipStream_t st) {
  if (max_items == 0) return;
  hipLaunchKernelGGL(k_item_desc, dim3((max_items + 255) / 256), dim3(256),
                     0, st, g, offsets, counters, extra, busy, tile_chunks,
                     chunk, desc, max_items);
}

template <typename R>
void launch_zero_idle(const Geo& g, const uint32_t* counters,
                      const uint32_t* idle, void* planes, hipStream_t st) {
  if (g.ntiles <= 0) return;
  hipLaunchKernelGGL(k_zero_idle<R>, dim3((unsigned)g.ntiles), dim3(256), 0,
                     st, g, counters, idle, (cplx<R>*)planes);
}

template <typename R>
void launch_zero_idle_batch(const GridJob<R>* jobs, int njobs,
                            uint64_t total_tiles, hipStream_t st) {
  if (total_tiles == 0) return;
  hipLaunchKernelGGL(k_zero_idle_batch<R>, dim3((unsigned)total_tiles),
                     dim3(256), 0, st, jobs, njobs);
}

template <typename R>
void launch_grid_merge(const Geo& g, const uint32_t* counters,
                       const uint32_t* split_list, const uint32_t* tile_chunks,
                       const uint32_t* tile_slot, const void* partials,
                       void* planes, int accumulate, uint32_t max_split,
                       void* tstore, const uint32_t* tslot, uint32_t tcap,
                       hipStream_t st) {
  constexpr unsigned kMergeParts = 4;
  hipLaunchKernelGGL(k_grid_merge<R>, dim3(max_split, kMergeParts), dim3(1024),
                     0, st, g,
                     counters, split_list, tile_chunks, tile_slot,
                     (const cplx<R>*)partials, (cplx<R>*)planes, accumulate,
                     (cplx<R>*)tstore, tslot, tcap);
}

template <typename R>
void launch_degrid_tiles(const Geo& g, const uint32_t* offsets,
                         uint32_t* counters, const uint2* extra,
                         const uint32_t* busy, const void* planes,
                         const void* records, uint32_t chunk,
                         void* vis_out, uint32_t max_items, int cus,
                         hipStream_t st) {
  WS_K_SWITCH(g.K, g.kern, (degrid_k<R, KK, KT>(g, offsets, counters,
                                                extra, busy, planes, records,
                                                chunk, vis_out, max_items,
                                                cus, st)));
}

#undef WS_K_SWITCH
#undef WS_KT_SWITCH

size_t degrid_lds_bytes(int T, int K, int elem_bytes) {
  const int W = T + K - 1;
  return (size_t)W * W * elem_bytes;
}

#define WS_INST(R)                                                          \
  template void launch_grid_tiles<R>(const GridJob<R>&, uint32_t, int,     \
                                     hipStream_t);                         \
  template void launch_grid_batch<R>(const GridJob<R>*, int, int, int,     \
                                     size_t, uint32_t*, uint32_t, int,     \
                                     hipStream_t);                         \
  template void launch_zero_idle<R>(const Geo&, const uint32_t*,           \
                                    const uint32_t*, void*, hipStream_t);  \
  template void launch_zero_idle_batch<R>(const GridJob<R>*, int, uint64_t, \
                                          hipStream_t);                    \
  template void launch_grid_merge<R>(const Geo&, const uint32_t*,          \
                                     const uint32_t*, const uint32_t*,     \
                                     const uint32_t*, const void*, void*,  \
                                     int, uint32_t, void*,                 \
                                     const uint32_t*, uint32_t,            \
                                     hipStream_t);                         \
  template void launch_degrid_tiles<R>(                                    \
      const Geo&, const uint32_t*, uint32_t*, const uint2*,                \
      const uint32_t*, const void*, const void*, uint32_t, void*,          \
      uint32_t, int, hipStream_t);
WS_INST(float)
WS_INST(double)
#undef WS_INST

}  // namespace ws
