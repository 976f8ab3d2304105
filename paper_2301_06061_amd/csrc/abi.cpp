// C ABI of libwstack.so: argument checks, workspace layout, plan state and
// the launch sequences of the four imaging steps (Sec. 2: gridding, FFT,
// phase correction and plane reduction) and of degridding.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "wstack.h"
#include "ws_kernels.h"

using namespace ws;

namespace {

thread_local std::string g_last_error;

ws_status fail(ws_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Grid edge limit: the record packs each cell index in 16 bits (with a
// bias of 64), and a 32768^2 FP32 plane is already 8.6 GB.
constexpr int kMaxN = 32768;
// Largest column length transformed in one pass (whole column blocks in
// LDS); longer columns use the four-step transform.
constexpr int kOnePassCols = 4096;
// Largest row length of the fused row-transform + screen kernels.
constexpr int kFusedRows = 4096;
constexpr int kMinN = 16;
constexpr int kMaxSupport = 15;
constexpr int64_t kMaxVis = (int64_t(1) << 31) - 1;
// Partition binning: level-1 histogram of at most this many buckets, and
// buckets of at most this many keys (64 KB of LDS each).
constexpr int kPartMaxBuckets = 16384;
constexpr int kPartMaxSpan = 16384;

enum PlaneState { kEmpty = 0, kGridded = 1, kTransformed = 2 };

// Derived sizes of a parameter set.
struct Layout {
  int T;
  uint32_t chunk;
  uint32_t chunk_degrid;
  int elem;
  int64_t ntiles;
  int64_t nkeys;
  uint32_t max_slots;
  uint32_t max_extra;
  size_t planes_bytes;
  // binning: WS_BINNING_PARTITION or WS_BINNING_HASHED (resolved)
  int binning;
  uint32_t part_buckets, part_span;  // partition: buckets and keys each
  // Busy-tile store of the one-call path (FP32, 4096-row columns, tile
  // edge 64, fused rows): tiles with records are gridded into slots of
  // their own and the column transform reads them contiguously.
  bool tstore;
  int64_t tstore_slots;
  // workspace offsets
  size_t o_tw_u, o_tw_v, o_corr, o_counts, o_sums, o_keyrank, o_rec, o_chunks,
      o_slot, o_counters, o_split, o_extra, o_busy, o_idle, o_copies, o_desc,
      o_strips, o_partials, o_scratch, o_rowscratch, o_clean, o_p_hist1, o_p_hist1x,
      o_p_btot, o_p_bounds, o_p_seg, o_p_rec1, o_p_keys, o_p_chunk0, o_p_rank2,
      o_p_hist2, o_p_hist2x, o_tstore, o_tslot, o_zero, total;
};

ws_status check_params(const ws_params* p) {
  if (p == nullptr) return fail(WS_INVALID_ARG, "params is NULL");
  if (!pow2(p->nu) || !pow2(p->nv))
    return fail(WS_UNSUPPORTED_SIZE, "nu=%d, nv=%d: must be powers of two",
                p->nu, p->nv);
  if (p->nu < kMinN || p->nv < kMinN || p->nu > kMaxN || p->nv > kMaxN)
    return fail(WS_UNSUPPORTED_SIZE, "nu=%d, nv=%d: supported range [%d, %d]",
                p->nu, p->nv, kMinN, kMaxN);
  if (p->nw < 1) return fail(WS_INVALID_ARG, "nw=%d: need >= 1", p->nw);
  if (p->support < 1 || p->support > kMaxSupport || (p->support % 2) == 0)
    return fail(WS_UNSUPPORTED_SIZE, "support=%d: must be odd in [1, %d]",
                p->support, kMaxSupport);
  if (!(p->fov_l > 0) || !(p->fov_m > 0) || !std::isfinite(p->fov_l) ||
      !std::isfinite(p->fov_m))
    return fail(WS_INVALID_ARG, "fov must be finite and > 0");
  const double c2 = 0.25 * (p->fov_l * p->fov_l + p->fov_m * p->fov_m);
  if (!(c2 < 1.0))
    return fail(WS_INVALID_ARG, "field of view reaches past the horizon");
  if (!std::isfinite(p->w_min) || !std::isfinite(p->w_max))
    return fail(WS_INVALID_ARG, "w range must be finite");
  if (p->nw > 1 && !(p->w_max > p->w_min))
    return fail(WS_INVALID_ARG, "w_max must exceed w_min when nw > 1");
  if (p->nw == 1 && p->w_max < p->w_min)
    return fail(WS_INVALID_ARG, "w_max < w_min");
  if (!std::isfinite(p->sigma))
    return fail(WS_INVALID_ARG, "sigma must be finite");
  if (p->kernel != WS_KERNEL_GAUSS && p->kernel != WS_KERNEL_ES)
    return fail(WS_INVALID_ARG,
                "kernel=%d: use WS_KERNEL_GAUSS or WS_KERNEL_ES", p->kernel);
  if (!std::isfinite(p->beta) || p->beta > 200.0)
    return fail(WS_INVALID_ARG, "beta must be finite and <= 200");
  if (p->correct != 0 && p->correct != 1)
    return fail(WS_INVALID_ARG, "correct=%d: use 0 or 1", p->correct);
  if (p->binning != WS_BINNING_AUTO && p->binning != WS_BINNING_PARTITION &&
      p->binning != WS_BINNING_HASHED)
    return fail(WS_INVALID_ARG, "binning=%d: use WS_BINNING_AUTO, "
                "WS_BINNING_PARTITION or WS_BINNING_HASHED", p->binning);
  if (p->precision != WS_FP32 && p->precision != WS_FP64)
    return fail(WS_INVALID_ARG, "precision=%d: use WS_FP32 or WS_FP64",
                p->precision);
  if (p->tile != 0) {
    if (!pow2(p->tile) || p->tile < 16 || p->tile > 64)
      return fail(WS_UNSUPPORTED_SIZE, "tile=%d: power of two in [16, 64]",
                  p->tile);
    if (p->tile > p->nu || p->tile > p->nv)
      return fail(WS_UNSUPPORTED_SIZE, "tile=%d larger than the grid",
                  p->tile);
    if (p->tile <= p->support - 1)
      return fail(WS_UNSUPPORTED_SIZE, "tile=%d must exceed support-1",
                  p->tile);
  }
  if (!fft_supported(p->nu, p->precision == WS_FP64 ? 16 : 8))
    return fail(WS_UNSUPPORTED_SIZE,
                "nu=%d: a quarter row must fit one workgroup's LDS", p->nu);
  if (p->chunk < 0 || p->chunk > (1 << 24))
    return fail(WS_INVALID_ARG, "chunk=%d out of range", p->chunk);
  const int64_t cells = (int64_t)p->nu * p->nv;
  if (p->nw > (int64_t(1) << 40) / cells)
    return fail(WS_UNSUPPORTED_SIZE, "plane stack too large");
  if (p->correct) {
    // The correction divides by the kernel's transform, which must stay
    // positive out to the highest pixel frequency, |f| = 1/2 cycle per cell
    // (psi is even).  Checked on 257 frequencies; a kernel wide enough for
    // a sign change of psi inside |f| <= 1/2 (a broad truncated Gaussian,
    // a small beta) shows it on this grid.
    const double sigma = p->sigma > 0 ? p->sigma : p->support / 7.0;
    const double beta = p->beta > 0 ? p->beta : 2.3 * p->support;
    const double psi0 = kernel_transform(p->kernel, p->support,
                                         1.0 / (2.0 * sigma * sigma), beta,
                                         0.0);
    for (int i = 0; i <= 256; ++i) {
      const double psi = kernel_transform(p->kernel, p->support,
                                          1.0 / (2.0 * sigma * sigma), beta,
                                          0.5 * i / 256.0);
      if (!(psi > 1e-12 * psi0))
        return fail(WS_INVALID_ARG,
                    "grid correction: the kernel's transform is not positive "
                    "at f = %.4f cycles per cell (psi = %g)", 0.5 * i / 256.0,
                    psi);
    }
  }
  return WS_OK;
}

ws_status make_layout(const ws_params* p, int64_t max_vis, Layout* L) {
  ws_status st = check_params(p);
  if (st != WS_OK) return st;
  if (max_vis < 1 || max_vis > kMaxVis)
    return fail(WS_INVALID_ARG, "max_vis=%lld: need 1 <= max_vis < 2^31",
                (long long)max_vis);
  const int nmin = p->nu < p->nv ? p->nu : p->nv;
  L->T = p->tile != 0 ? p->tile : (nmin < 64 ? nmin : 64);
  if (L->T <= p->support - 1)
    return fail(WS_UNSUPPORTED_SIZE, "grid %d too small for support %d", nmin,
                p->support);
  L->chunk = p->chunk != 0 ? (uint32_t)p->chunk : 4096u;
  L->chunk_degrid = p->chunk != 0 ? (uint32_t)p->chunk : 4096u;
  L->elem = p->precision == WS_FP64 ? 16 : 8;
  const int64_t tu = p->nu / L->T, tv = p->nv / L->T;
  L->ntiles = tu * tv * p->nw;
  L->nkeys = L->ntiles * kRegions;
  if (L->nkeys >= (int64_t)0xFFFFFFF0ll)
    return fail(WS_UNSUPPORTED_SIZE, "too many bins (%lld)",
                (long long)L->nkeys);
  // Partition buckets: a plane and G tile rows (G a power of two dividing
  // tiles_v), the fewest rows that keep the level-1 histogram within 64 KB
  // of LDS; the level-2 histogram (the keys of one bucket) must fit too.
  {
    int64_t G = 1;
    while (p->nw * (tv / G) > kPartMaxBuckets && G < tv) G *= 2;
    const int64_t buckets = p->nw * (tv / G);
    const int64_t span = G * tu * kRegions;
    const bool fits = buckets <= kPartMaxBuckets && span <= kPartMaxSpan;
    if (p->binning == WS_BINNING_PARTITION && !fits)
      return fail(WS_UNSUPPORTED_SIZE,
                  "partition binning: %lld buckets of %lld keys exceed the "
                  "LDS histograms (<= %d buckets, <= %d keys)",
                  (long long)buckets, (long long)span, kPartMaxBuckets,
                  kPartMaxSpan);
    L->binning = (p->binning == WS_BINNING_HASHED || !fits)
                     ? WS_BINNING_HASHED : WS_BINNING_PARTITION;
    L->part_buckets = (uint32_t)buckets;
    L->part_span = (uint32_t)span;
  }
  int64_t slots = 2 * max_vis / L->chunk + 64;
  if (slots > 4096) slots = 4096;
  L->max_slots = (uint32_t)slots;
  // Further work items beyond one per tile: at most max_slots when
  // gridding (split tiles hold scratch slots), at most max_vis / chunk when
  // degridding (each record is read by one tile).
  const int64_t ex = max_vis / L->chunk_degrid + 2;
  L->max_extra = (uint32_t)(ex > slots ? ex : slots);
  L->planes_bytes = (size_t)p->nw * p->nv * p->nu * L->elem;
  const size_t A = 256;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes, A);
    return at;
  };
  const int64_t nscan = L->nkeys > L->ntiles ? L->nkeys : L->ntiles;
  L->o_tw_u = take((size_t)p->nu * L->elem);
  L->o_tw_v = take((size_t)p->nv * L->elem);
  // Grid-correction factors (u axis, then v axis), FP64.
  L->o_corr = take((size_t)(p->nu + p->nv) * 8);
  // Key counts, scanned in place into key offsets (+ the total).
  L->o_counts = take((size_t)(L->nkeys + 1) * 4);
  const bool part = L->binning == WS_BINNING_PARTITION;
  // kCountCopies copies of the key counts, turned into per-copy offsets
  // (hashed binning only).
  L->o_copies = take(part ? 0 : (size_t)kCountCopies * L->nkeys * 4);
  const int64_t pblocks = partition_blocks(max_vis, L->elem);
  const int64_t pscan = (int64_t)L->part_buckets * pblocks;
  L->o_sums = take((size_t)(scan_sums_len(nscan) + 1) * 4);
  // Partition: level-1 histograms (block-major, then bucket-major and
  // scanned), records and keys in bucket order, chunk starts, level-2
  // ranks and histograms.
  L->o_p_hist1 = take(part ? (size_t)pscan * 4 : 0);
  L->o_p_hist1x = take(part ? (size_t)pscan * 4 : 0);
  L->o_p_btot = take(part ? (size_t)pblocks * 4 : 0);
  L->o_p_bounds = take(part ? (size_t)(L->part_buckets + 1) * 4 : 0);
  L->o_p_seg = take(part ? (size_t)64 * L->part_buckets * 4 : 0);
  L->o_p_rec1 = take(part ? (size_t)max_vis *
                                (L->elem == 16 ? sizeof(Record<double>)
                                               : sizeof(Record<float>))
                          : 0);
  L->o_p_keys = take(part ? (size_t)max_vis * 4 : 0);
  L->o_p_chunk0 = take(part ? (size_t)(L->part_buckets + 1) * 4 : 0);
  L->o_p_rank2 = take(part ? (size_t)max_vis * 4 : 0);
  const size_t h2 = part ? (size_t)partition_chunks(max_vis, L->part_buckets,
                                                     L->elem) *
                               L->part_span * 4
                         : 0;
  L->o_p_hist2 = take(h2);
  L->o_p_hist2x = take(h2);
  L->o_keyrank = take((size_t)max_vis * 8);
  L->o_rec = take((size_t)max_vis *
                  (L->elem == 16 ? sizeof(Record<double>)
                                 : sizeof(Record<float>)));
  L->o_chunks = take((size_t)(L->ntiles + 1) * 4);
  L->o_slot = take((size_t)L->ntiles * 4);
  L->o_counters = take(64);
  L->o_split = take((size_t)(L->max_slots / 2 + 1) * 4);
  L->o_extra = take((size_t)L->max_extra * 8);
  L->o_busy = take((size_t)L->ntiles * 4);
  // One descriptor per gridding work item (every tile, every extra chunk).
  L->o_desc = take((size_t)(L->ntiles + L->max_extra + 1) * kDescWords * 4);
  L->o_idle = take((size_t)L->ntiles * 4);
  // Column strips (T columns of one plane) that some gridding call since
  // the reset wrote records into.
  L->o_strips = take((size_t)p->nw * (p->nu / L->T) * 4);
  L->o_partials = take((size_t)L->max_slots * L->T * L->T * L->elem);
  // One plane of scratch for the natural-order output of ws_fft_planes
  // when columns use the four-step transform.
  L->o_scratch = take(p->nv > kOnePassCols
                          ? (size_t)p->nu * p->nv * L->elem : (size_t)0);
  // Scratch rows of the 4-way split row transform (rows too long for two
  // half-length LDS transforms).
  L->o_rowscratch = take(fft_row_scratch_bytes(p->nu, L->elem));
  // Minor-cycle state and its per-block argmax slots.
  L->o_clean = take(sizeof(CleanState) + kCleanMaxSlots * sizeof(CleanSlot));
  // Busy-tile store: T x T slots for half the tiles at most (tiles with
  // records beyond that stay in the stack; each visibility is read by at
  // most four tiles), and the slot of every tile.
  L->tstore = L->elem == 8 && p->nv == 4096 && L->T == 64 && p->nu >= 512 &&
              p->nu <= kFusedRows;
  L->tstore_slots =
      L->tstore ? std::max<int64_t>(
                      1, std::min<int64_t>(L->ntiles / 2, 4 * max_vis))
                : 0;
  L->o_tstore = take((size_t)L->tstore_slots * L->T * L->T * L->elem);
  L->o_tslot = take(L->tstore ? (size_t)L->ntiles * 4 : (size_t)0);
  // 256 bytes of zeros: where the column transform's loads of rows
  // without records go.
  L->o_zero = take(256);
  L->total = o;
  return WS_OK;
}

}  // namespace

struct ws_plan {
  ws_params p;
  int64_t max_vis;
  Layout L;
  Geo g;
  void* planes;
  unsigned char* work;
  hipStream_t stream;
  int state;
  int device;
  int cus;  // compute units of the device (sizes persistent launches)
  // profiling
  bool profile;
  struct Pending {
    int id;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<const char*> names;
  std::vector<double> ms;
  std::vector<int64_t> launches;

  template <typename T>
  T* w(size_t off) {
    return reinterpret_cast<T*>(work + off);
  }
};

namespace {

int kernel_id(ws_plan* pl, const char* name) {
  for (size_t i = 0; i < pl->names.size(); ++i)
    if (std::strcmp(pl->names[i], name) == 0) return (int)i;
  pl->names.push_back(name);
  pl->ms.push_back(0.0);
  pl->launches.push_back(0);
  return (int)pl->names.size() - 1;
}

// Runs one launcher; when profiling, brackets it with events on the stream.
template <class F>
ws_status launch(ws_plan* pl, const char* name, F&& f) {
  hipEvent_t a = nullptr, b = nullptr;
  if (pl->profile) {
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
      return fail(WS_HIP_ERROR, "hipEventCreate failed");
    hipEventRecord(a, pl->stream);
  }
  f();
  hipError_t e = hipGetLastError();
  if (pl->profile) {
    hipEventRecord(b, pl->stream);
    pl->pending.push_back({kernel_id(pl, name), a, b});
  }
  if (e != hipSuccess)
    return fail(WS_HIP_ERROR, "%s: launch failed: %s", name,
                hipGetErrorString(e));
  return WS_OK;
}

#define WS_TRY(expr)                 \
  do {                               \
    ws_status _s = (expr);           \
    if (_s != WS_OK) return _s;      \
  } while (0)

Geo make_geo(const ws_params* p, const Layout& L) {
  Geo g{};
  g.nu = p->nu;
  g.nv = p->nv;
  g.nw = p->nw;
  g.K = p->support;
  g.h = (p->support - 1) / 2;
  g.T = L.T;
  g.tiles_u = p->nu / L.T;
  g.tiles_v = p->nv / L.T;
  g.ntiles = (int)L.ntiles;
  g.fov_l = p->fov_l;
  g.fov_m = p->fov_m;
  g.w_min = p->w_min;
  if (p->nw == 1) {
    g.dw = 1.0;
    g.w0 = 0.5 * (p->w_min + p->w_max);
  } else {
    g.dw = (p->w_max - p->w_min) / p->nw;
    g.w0 = p->w_min + 0.5 * g.dw;
  }
  g.dl = p->fov_l / p->nu;
  g.dm = p->fov_m / p->nv;
  const double sigma = p->sigma > 0 ? p->sigma : p->support / 7.0;
  g.inv2s2 = 1.0 / (2.0 * sigma * sigma);
  g.kappa = (float)(1.4426950408889634074 / (2.0 * sigma * sigma));
  g.kern = p->kernel;
  g.es_beta = p->beta > 0 ? p->beta : 2.3 * p->support;
  g.es_zs = 2.0 / p->support;
  g.es_beta2 = (float)(g.es_beta * 1.4426950408889634074);
  g.es_zs_f = (float)g.es_zs;
  if (p->kernel == WS_KERNEL_ES) {
    // c = 1 / (integral of phi)^2: the continuous 2-D kernel integrates to
    // one, as the Gaussian's 1 / (2 pi sigma^2) does.
    const double psi0 = kernel_transform(g.kern, g.K, g.inv2s2, g.es_beta,
                                         0.0);
    g.cnorm = 1.0 / (psi0 * psi0);
  } else {
    g.cnorm = 1.0 / (2.0 * M_PI * sigma * sigma);
  }
  g.corr = nullptr;  // set by init_plan when the plan corrects
  return g;
}

template <typename R>
ws_status zero_planes(ws_plan* pl) {
  const int64_t n = (int64_t)pl->p.nw * pl->p.nv * pl->p.nu;
  return launch(pl, "fill_zero",
                [&] { launch_fill_zero<R>(pl->planes, n, pl->stream); });
}

// Binning shared by gridding and degridding: counts, offsets, records and
// the per-tile work items.  Returns the grid size bound for the item kernel.
// For gridding, `strips` (cleared first when clear_strips) gets a mark for
// every column strip that holds a tile with records.
VisSource flat_source(const double* uvw, const void* vis,
                      const float* weight) {
  VisSource s{};
  s.uvw = uvw;
  s.vis = vis;
  s.weight = weight;
  s.rows = 0;
  return s;
}

template <typename R>
ws_status bin_records(ws_plan* pl, int64_t m, const VisSource& src,
                      int degrid, int64_t* n_dropped, uint32_t* max_items,
                      uint32_t* strips = nullptr, bool clear_strips = false,
                      void* vis_out = nullptr, uint32_t* tslot = nullptr) {
  const Layout& L = pl->L;
  const Geo& g = pl->g;
  hipStream_t st = pl->stream;
  uint32_t* counts = pl->w<uint32_t>(L.o_counts);
  uint32_t* sums = pl->w<uint32_t>(L.o_sums);
  uint2* keyrank = pl->w<uint2>(L.o_keyrank);
  uint32_t* chunks = pl->w<uint32_t>(L.o_chunks);
  uint32_t* slot = pl->w<uint32_t>(L.o_slot);
  uint32_t* counters = pl->w<uint32_t>(L.o_counters);
  uint32_t* split = pl->w<uint32_t>(L.o_split);
  const uint32_t chunk = degrid ? L.chunk_degrid : L.chunk;
  uint32_t* copies = pl->w<uint32_t>(L.o_copies);
  const uint32_t nkeys = (uint32_t)L.nkeys;
  const bool part = L.binning == WS_BINNING_PARTITION;
  WS_TRY(launch(pl, "zero_counts", [&] {
    if (!part) launch_zero_u32(copies, kCountCopies * L.nkeys, st);
    launch_zero_u32(counters, 16, st);
    if (strips != nullptr && clear_strips)
      launch_zero_u32(strips, (int64_t)g.nw * g.tiles_u, st);
  }));
  if (part) {
    PartWork w;
    w.nbuckets = L.part_buckets;
    w.span = L.part_span;
    w.keyrank = keyrank;
    w.hist1 = pl->w<uint32_t>(L.o_p_hist1);
    w.hist1x = pl->w<uint32_t>(L.o_p_hist1x);
    w.btot = pl->w<uint32_t>(L.o_p_btot);
    w.hist2x = pl->w<uint32_t>(L.o_p_hist2x);
    w.bounds = pl->w<uint32_t>(L.o_p_bounds);
    w.seg = pl->w<uint32_t>(L.o_p_seg);
    w.sums = sums;
    w.rec1 = pl->work + L.o_p_rec1;
    w.keys = pl->w<uint32_t>(L.o_p_keys);
    w.chunk0 = pl->w<uint32_t>(L.o_p_chunk0);
    w.rank2 = pl->w<uint32_t>(L.o_p_rank2);
    w.hist2 = pl->w<uint32_t>(L.o_p_hist2);
    w.offsets = counts;
    w.rec = pl->work + L.o_rec;
    auto* drop = reinterpret_cast<unsigned long long*>(n_dropped);
    WS_TRY(launch(pl, "part_count1", [&] {
      launch_part_count1<R>(g, src, m, w, drop, st);
    }));
    WS_TRY(launch(pl, "part_scan1", [&] { launch_part_scan1<R>(m, w, st); }));
    WS_TRY(launch(pl, "part_scatter1", [&] {
      launch_part_scatter1<R>(g, src, m, w, degrid, vis_out, st);
    }));
    WS_TRY(launch(pl, "part_count2", [&] {
      launch_part_count2<R>(m, w, st);
    }));
    WS_TRY(launch(pl, "part_scan2", [&] { launch_part_scan2<R>(m, w, st); }));
    WS_TRY(launch(pl, "part_scatter2", [&] {
      launch_part_scatter2<R>(m, w, st);
    }));
  } else {
    WS_TRY(launch(pl, "bin_count", [&] {
      launch_bin_count(g, src, m, copies, nkeys, keyrank,
                       reinterpret_cast<unsigned long long*>(n_dropped), st);
    }));
    WS_TRY(launch(pl, "scan_keys", [&] {
      launch_fold_copies(copies, nkeys, counts, st);
      launch_exclusive_scan(counts, counts, L.nkeys, sums, st);
      launch_copy_offsets(copies, nkeys, counts, st);
    }));
    WS_TRY(launch(pl, "bin_scatter", [&] {
      launch_bin_scatter<R>(g, src, m, keyrank, copies, nkeys,
                            pl->work + L.o_rec, degrid, vis_out, st);
    }));
  }
  WS_TRY(launch(pl, "tile_work", [&] {
    launch_tile_work(g, counts, degrid, chunk, chunks, slot, counters, split,
                     L.max_slots, pl->w<uint2>(L.o_extra), L.max_extra,
                     pl->w<uint32_t>(L.o_busy), pl->w<uint32_t>(L.o_idle),
                     strips, tslot, st);
  }));
  // Items: one per tile plus the further chunks of split tiles.
  const int64_t reads = degrid ? m : 4 * m;
  int64_t extra = (reads + chunk - 1) / chunk + 1;
  if (extra > L.max_extra) extra = L.max_extra;
  *max_items = (uint32_t)(L.ntiles + extra);
  if (!degrid) {
    // Extra items are capped by max_extra, so every item has a slot.
    WS_TRY(launch(pl, "item_desc", [&] {
      launch_item_desc(g, counts, counters, pl->w<uint2>(L.o_extra),
                       pl->w<uint32_t>(L.o_busy), chunks, chunk,
                       pl->w<uint32_t>(L.o_desc),
                       (uint32_t)(L.ntiles + L.max_extra), st);
    }));
  }
  return WS_OK;
}

bool lazy_ok(const ws_plan* pl);
bool tstore_ok(const ws_plan* pl);
bool marked_ok(const ws_plan* pl);

// With `ts`, finished tiles go to the busy-tile store.
template <typename R>
GridJob<R> make_job(ws_plan* pl, int accumulate, bool ts = false) {
  const Layout& L = pl->L;
  GridJob<R> j;
  j.g = pl->g;
  j.pitch = grid_lds_pitch(L.T, pl->p.support);
  j.offsets = pl->w<uint32_t>(L.o_counts);
  j.counters = pl->w<uint32_t>(L.o_counters);
  j.extra = pl->w<uint2>(L.o_extra);
  j.busy = pl->w<uint32_t>(L.o_busy);
  j.idle = pl->w<uint32_t>(L.o_idle);
  j.tile_chunks = pl->w<uint32_t>(L.o_chunks);
  j.tile_slot = pl->w<uint32_t>(L.o_slot);
  j.rec = pl->w<Record<R>>(L.o_rec);
  j.desc = pl->w<uint32_t>(L.o_desc);
  j.chunk = L.chunk;
  j.planes = static_cast<cplx<R>*>(pl->planes);
  j.partials = pl->w<cplx<R>>(L.o_partials);
  j.accumulate = accumulate;
  j.zero_idle = lazy_ok(pl) ? 0 : 1;
  j.tstore = ts ? pl->w<cplx<R>>(L.o_tstore) : nullptr;
  j.tslot = ts ? pl->w<uint32_t>(L.o_tslot) : nullptr;
  j.tcap = ts ? (uint32_t)L.tstore_slots : 0u;
  return j;
}

template <typename R>
ws_status merge_impl(ws_plan* pl, int acc, bool ts = false) {
  const Layout& L = pl->L;
  return launch(pl, "grid_merge", [&] {
    launch_grid_merge<R>(pl->g, pl->w<uint32_t>(L.o_counters),
                         pl->w<uint32_t>(L.o_split),
                         pl->w<uint32_t>(L.o_chunks),
                         pl->w<uint32_t>(L.o_slot), pl->work + L.o_partials,
                         pl->planes, acc, L.max_slots / 2 + 1,
                         ts ? pl->work + L.o_tstore : nullptr,
                         ts ? pl->w<uint32_t>(L.o_tslot) : nullptr,
                         (uint32_t)L.tstore_slots, pl->stream);
  });
}

// With `lazy` (a first call whose stack only the one-call imaging path
// will read), tiles without records are not zeroed; with `ts` as well,
// tiles with records go to the busy-tile store instead of the stack.
template <typename R>
ws_status grid_impl(ws_plan* pl, int64_t m, const VisSource& src,
                    int64_t* n_dropped, bool lazy = false, bool ts = false) {
  uint32_t max_items = 0;
  const int acc = pl->state == kGridded ? 1 : 0;
  ts = ts && lazy && !acc;
  WS_TRY(bin_records<R>(pl, m, src, 0, n_dropped, &max_items,
                        pl->w<uint32_t>(pl->L.o_strips), !acc, nullptr,
                        ts ? pl->w<uint32_t>(pl->L.o_tslot) : nullptr));
  const GridJob<R> j = make_job<R>(pl, acc, ts);
  if (!acc && !lazy) {
    // First call since the reset: tiles without records get their zeros.
    WS_TRY(launch(pl, "zero_idle", [&] {
      launch_zero_idle<R>(pl->g, j.counters, j.idle, pl->planes, pl->stream);
    }));
  }
  WS_TRY(launch(pl, "grid_tiles", [&] {
    launch_grid_tiles<R>(j, max_items, pl->cus, pl->stream);
  }));
  WS_TRY(merge_impl<R>(pl, acc, ts));
  pl->state = kGridded;
  return WS_OK;
}

// Column transform of every plane: one pass for columns up to
// kOnePassCols, else the four-step transform, which leaves the rows in the
// transposed order described by the returned geometry.
// With `strips` (marks of the column strips that hold records), strips
// without marks are skipped: gridding left them zero, and so is their
// transform.
template <typename R>
ws_status cols_impl(ws_plan* pl, int sign, Geo* gout,
                    const uint32_t* strips = nullptr,
                    const uint32_t* tiles = nullptr, bool ts = false) {
  const ws_params& p = pl->p;
  bool ok = true;
  Geo g = pl->g;
  if (p.nv <= kOnePassCols) {
    WS_TRY(launch(pl, "fft_cols", [&] {
      ok = launch_fft_cols<R>(pl->planes, p.nv, p.nu, p.nw,
                              pl->work + pl->L.o_tw_v, sign, strips, g.T,
                              tiles, ts ? pl->work + pl->L.o_tstore : nullptr,
                              ts ? pl->w<uint32_t>(pl->L.o_tslot) : nullptr,
                              (uint32_t)pl->L.tstore_slots, pl->stream);
    }));
  } else {
    WS_TRY(launch(pl, "fft_cols4", [&] {
      ok = launch_fft_cols4<R>(pl->planes, p.nv, p.nu, p.nw,
                               pl->work + pl->L.o_tw_v, sign, strips, g.T,
                               tiles, pl->work + pl->L.o_zero, pl->stream);
    }));
    int lg = 0;
    while ((1 << lg) < p.nv) ++lg;
    g.perm_n1 = 1 << (lg / 2);
    g.perm_n2 = p.nv / g.perm_n1;
  }
  if (!ok) return fail(WS_UNSUPPORTED_SIZE, "no column FFT for nv=%d", p.nv);
  *gout = g;
  return WS_OK;
}

// With `strips`, samples of unmarked column strips are taken as zero.
template <typename R>
ws_status rows_impl(ws_plan* pl, int sign, const uint32_t* strips = nullptr) {
  const ws_params& p = pl->p;
  bool ok = true;
  WS_TRY(launch(pl, "fft_rows", [&] {
    ok = launch_fft_rows<R>(pl->planes, p.nu, (int64_t)p.nw * p.nv,
                            pl->work + pl->L.o_tw_u, sign,
                            pl->work + pl->L.o_rowscratch, strips, p.nv,
                            pl->stream);
  }));
  if (!ok) return fail(WS_UNSUPPORTED_SIZE, "no row FFT for nu=%d", p.nu);
  return WS_OK;
}

template <typename R>
ws_status fft_impl(ws_plan* pl, int sign) {
  const ws_params& p = pl->p;
  WS_TRY(rows_impl<R>(pl, sign));
  Geo g;
  WS_TRY(cols_impl<R>(pl, sign, &g));
  if (g.perm_n1 != 0) {
    // Natural row order for the caller: each plane through the scratch.
    const size_t plane = (size_t)p.nu * p.nv * sizeof(cplx<R>);
    for (int k = 0; k < p.nw; ++k) {
      unsigned char* pk = static_cast<unsigned char*>(pl->planes) + k * plane;
      WS_TRY(launch(pl, "unpermute_rows", [&] {
        launch_unpermute_rows<R>(pk, pl->work + pl->L.o_scratch, g,
                                 pl->stream);
        hipMemcpyAsync(pk, pl->work + pl->L.o_scratch, plane,
                       hipMemcpyDeviceToDevice, pl->stream);
      }));
    }
  }
  return WS_OK;
}

// The stack holds what the gridding calls since the reset wrote, so the
// column strips they never reached are skipped.
// With `lazy`, tiles without records were never written (their cells are
// taken as zero from the per-tile record counts); with `ts` as well, the
// tiles with records are in the busy-tile store.
// With `marked` (the one-call path beyond 4096), tiles without records
// were never written either: the column transform reads by tile record
// counts and the row transform takes unmarked strips as zero.
template <typename R>
ws_status image_impl(ws_plan* pl, void* image, bool lazy = false,
                     bool ts = false, bool marked = false) {
  const ws_params& p = pl->p;
  Geo g;
  WS_TRY(cols_impl<R>(pl, +1, &g, pl->w<uint32_t>(pl->L.o_strips),
                      lazy || marked ? pl->w<uint32_t>(pl->L.o_chunks)
                                     : nullptr,
                      lazy && ts));
  if (p.nu <= kFusedRows) {
    bool ok = true;
    WS_TRY(launch(pl, "row_screen_sum", [&] {
      ok = launch_row_screen_sum<R>(pl->planes, image, g,
                                    pl->work + pl->L.o_tw_u,
                                    pl->w<uint32_t>(pl->L.o_strips),
                                    pl->stream);
    }));
    if (!ok) return fail(WS_UNSUPPORTED_SIZE, "no fused row FFT for nu=%d",
                         p.nu);
    return WS_OK;
  }
  WS_TRY(rows_impl<R>(pl, +1,
                      marked ? pl->w<uint32_t>(pl->L.o_strips) : nullptr));
  return launch(pl, "wcorrect", [&] {
    launch_wcorrect<R>(pl->planes, image, g, pl->stream);
  });
}

template <typename R>
ws_status degrid_impl(ws_plan* pl, const void* image, int image_is_real,
                      int64_t m, const double* uvw, const float* weight,
                      void* vis_out) {
  const ws_params& p = pl->p;
  const Layout& L = pl->L;
  Geo g = pl->g;
  if (p.nu <= kFusedRows) {
    bool ok = true;
    WS_TRY(launch(pl, "screen_row_bcast", [&] {
      ok = launch_screen_row_bcast<R>(image, image_is_real, pl->planes,
                                      pl->g, pl->work + L.o_tw_u, pl->stream);
    }));
    if (!ok) return fail(WS_UNSUPPORTED_SIZE, "no fused row FFT for nu=%d",
                         p.nu);
  } else {
    WS_TRY(launch(pl, "screen_bcast", [&] {
      launch_screen_bcast<R>(image, image_is_real, pl->planes, pl->g,
                             pl->stream);
    }));
    WS_TRY(rows_impl<R>(pl, -1));
  }
  WS_TRY(cols_impl<R>(pl, -1, &g));
  if (m == 0) return WS_OK;
  uint32_t max_items = 0;
  WS_TRY(bin_records<R>(pl, m, flat_source(uvw, nullptr, weight), 1,
                        nullptr, &max_items, nullptr, false, vis_out));
  WS_TRY(launch(pl, "degrid_tiles", [&] {
    launch_degrid_tiles<R>(g, pl->w<uint32_t>(L.o_counts),
                           pl->w<uint32_t>(L.o_counters),
                           pl->w<uint2>(L.o_extra),
                           pl->w<uint32_t>(L.o_busy), pl->planes,
                           pl->work + L.o_rec,
                           L.chunk_degrid, vis_out, max_items, pl->cus,
                           pl->stream);
  }));
  return WS_OK;
}

bool aligned(const void* p, size_t a) {
  return (reinterpret_cast<uintptr_t>(p) % a) == 0;
}

// Tiles without records may stay unwritten only where every later read
// knows them: one-pass columns with tile-wide blocks and the fused rows
// reading by strip marks (tile edge 64, rows of 512 or more).
bool lazy_ok(const ws_plan* pl) {
  return pl->g.T == 64 && pl->p.nv <= kOnePassCols && pl->p.nu >= 512 &&
         pl->p.nu <= kFusedRows;
}

// A first gridding call that only the fused imaging reads may put its
// tiles with records in the busy-tile store (where the layout has one).
bool tstore_ok(const ws_plan* pl) { return lazy_ok(pl) && pl->L.tstore; }

// Beyond 4096 the one-call path leaves the tiles without records
// unwritten too: the column transform (one-pass or the first four-step
// step) reads by tile record counts and skips unmarked strips, and the
// row transform (fused below 4096 columns, else by strip marks) takes the
// unmarked strips as zero.
bool marked_ok(const ws_plan* pl) {
  const ws_params& p = pl->p;
  return !lazy_ok(pl) && pl->g.T == 64 && p.nu >= 1024 &&
         (p.nu > kFusedRows || p.nv > kOnePassCols) &&
         (p.nu <= kFusedRows || fft_rows_can_mask(p.nu, pl->L.elem));
}

ws_status check_plan(ws_plan* pl) {
  if (pl == nullptr) return fail(WS_INVALID_ARG, "plan is NULL");
  if (hipSetDevice(pl->device) != hipSuccess)
    return fail(WS_HIP_ERROR, "hipSetDevice(%d) failed", pl->device);
  return WS_OK;
}

// Gridding and imaging of an empty plan in one pass over the stack (the
// one-call path); the plan is empty afterwards.
ws_status grid_image_impl(ws_plan* pl, int64_t m, const VisSource& src,
                          void* image, int64_t* n_dropped) {
  const bool lazy = lazy_ok(pl);
  const bool f64 = pl->p.precision == WS_FP64;
  // The plan is empty here (the call's contract), so the gridding is a
  // first call and may use the busy-tile store.
  const bool ts = tstore_ok(pl) && pl->state == kEmpty;
  const bool marked = marked_ok(pl) && pl->state == kEmpty;
  ws_status st =
      f64 ? grid_impl<double>(pl, m, src, n_dropped, lazy || marked, false)
          : grid_impl<float>(pl, m, src, n_dropped, lazy || marked, ts);
  if (st == WS_OK)
    st = f64 ? image_impl<double>(pl, image, lazy, false, marked)
             : image_impl<float>(pl, image, lazy, ts, marked);
  pl->state = kEmpty;
  return st;
}

// Checks of a baseline-major call and its source (pol_coeff is a host
// array of npol (re, im) pairs).
ws_status rows_source(ws_plan* pl, int64_t nrows, int32_t nchan,
                      int32_t npol, const double* uvw_m,
                      const double* freq_hz, const void* vis,
                      const float* weight, const double* pol_coeff,
                      VisSource* out, int64_t* m) {
  if (nrows < 0 || nchan < 1 || npol < 1 || npol > kMaxPol)
    return fail(WS_INVALID_ARG, "nrows=%lld, nchan=%d, npol=%d: need nrows "
                ">= 0, nchan >= 1, 1 <= npol <= %d", (long long)nrows, nchan,
                npol, kMaxPol);
  if (nrows > pl->max_vis / nchan)
    return fail(WS_WORKSPACE_TOO_SMALL,
                "nrows * nchan = %lld * %d exceeds max_vis=%lld",
                (long long)nrows, nchan, (long long)pl->max_vis);
  if (pol_coeff == nullptr) return fail(WS_INVALID_ARG, "pol_coeff is NULL");
  for (int p = 0; p < 2 * npol; ++p)
    if (!std::isfinite(pol_coeff[p]))
      return fail(WS_INVALID_ARG, "pol_coeff must be finite");
  *m = nrows * nchan;
  if (*m > 0 && (uvw_m == nullptr || freq_hz == nullptr || vis == nullptr))
    return fail(WS_INVALID_ARG, "uvw_m, freq_hz or vis is NULL");
  if (!aligned(uvw_m, 8) || !aligned(freq_hz, 8) || !aligned(weight, 4) ||
      !aligned(vis, pl->L.elem))
    return fail(WS_INVALID_ARG, "misaligned uvw_m, freq_hz, vis or weight");
  VisSource s{};
  s.uvw = uvw_m;
  s.vis = vis;
  s.weight = weight;
  s.rows = 1;
  s.nchan = nchan;
  s.npol = npol;
  s.freq = freq_hz;
  for (int p = 0; p < npol; ++p) {
    s.coef[p][0] = pol_coeff[2 * p];
    s.coef[p][1] = pol_coeff[2 * p + 1];
  }
  *out = s;
  return WS_OK;
}

ws_status check_vis_args(ws_plan* pl, int64_t m, const double* uvw,
                         const float* weight) {
  if (m < 0 || m > pl->max_vis)
    return fail(WS_WORKSPACE_TOO_SMALL,
                "m=%lld outside [0, max_vis=%lld]", (long long)m,
                (long long)pl->max_vis);
  if (m > 0 && uvw == nullptr) return fail(WS_INVALID_ARG, "uvw is NULL");
  if (!aligned(uvw, 8) || !aligned(weight, 4))
    return fail(WS_INVALID_ARG, "misaligned uvw or weight");
  return WS_OK;
}

}  // namespace

struct ws_batch {
  int n;
  std::vector<ws_plan*> plans;
  unsigned char* work;
  int precision;
  int K;
  int kern;
  size_t lds;
  hipStream_t stream;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

namespace {

size_t batch_jobs_bytes(int n) {
  return align_up((size_t)n * sizeof(GridJob<double>), 256);
}

template <typename R>
ws_status batch_image_impl(ws_batch* b, const int64_t* m,
                           const double* const* uvw, const void* const* vis,
                           const float* const* weight, void* const* images) {
  uint32_t items = 0;
  for (int i = 0; i < b->n; ++i) {
    ws_plan* pl = b->plans[i];
    pl->stream = b->stream;
    pl->state = kEmpty;
    uint32_t mi = 0;
    WS_TRY(bin_records<R>(pl, m[i],
                          flat_source(uvw[i], vis[i],
                                      weight ? weight[i] : nullptr),
                          0, nullptr, &mi, pl->w<uint32_t>(pl->L.o_strips),
                          true, nullptr,
                          tstore_ok(pl) ? pl->w<uint32_t>(pl->L.o_tslot)
                                        : nullptr));
    items += mi;
  }
  ws_plan* p0 = b->plans[0];
  uint32_t* queue = reinterpret_cast<uint32_t*>(b->work + batch_jobs_bytes(b->n));
  WS_TRY(launch(p0, "zero_counts", [&] { launch_zero_u32(queue, 1, b->stream); }));
  // As in ws_grid_image, plan by plan: where the imaging reads by tile
  // counts and strip marks, tiles without records are never written; the
  // other plans' idle tiles get their zeros (the batched zeroing kernel
  // skips the jobs that need none).
  bool all_lazy = true;
  for (int i = 0; i < b->n; ++i) all_lazy = all_lazy && lazy_ok(b->plans[i]);
  if (!all_lazy) {
    uint64_t tiles = 0;
    for (int i = 0; i < b->n; ++i) tiles += (uint64_t)b->plans[i]->g.ntiles;
    WS_TRY(launch(p0, "zero_idle", [&] {
      launch_zero_idle_batch<R>(reinterpret_cast<const GridJob<R>*>(b->work),
                                b->n, tiles, b->stream);
    }));
  }
  WS_TRY(launch(p0, "grid_batch", [&] {
    launch_grid_batch<R>(reinterpret_cast<const GridJob<R>*>(b->work), b->n,
                         b->K, b->kern, b->lds, queue, items, p0->cus,
                         b->stream);
  }));
  for (int i = 0; i < b->n; ++i) {
    ws_plan* pl = b->plans[i];
    WS_TRY(merge_impl<R>(pl, 0, tstore_ok(pl)));
    pl->state = kGridded;
    ws_status st = image_impl<R>(pl, images[i], lazy_ok(pl), tstore_ok(pl));
    pl->state = kEmpty;
    WS_TRY(st);
  }
  return WS_OK;
}

ws_status check_batch_args(ws_batch* b, const int64_t* m,
                           const double* const* uvw, const void* const* vis,
                           void* const* images) {
  if (b == nullptr) return fail(WS_INVALID_ARG, "batch is NULL");
  if (m == nullptr || uvw == nullptr || vis == nullptr || images == nullptr)
    return fail(WS_INVALID_ARG, "batch argument arrays must not be NULL");
  for (int i = 0; i < b->n; ++i) {
    ws_plan* pl = b->plans[i];
    if (m[i] < 0 || m[i] > pl->max_vis)
      return fail(WS_WORKSPACE_TOO_SMALL, "plan %d: m=%lld outside [0, %lld]",
                  i, (long long)m[i], (long long)pl->max_vis);
    if (m[i] > 0 && (uvw[i] == nullptr || vis[i] == nullptr))
      return fail(WS_INVALID_ARG, "plan %d: uvw or vis is NULL", i);
    if (images[i] == nullptr)
      return fail(WS_INVALID_ARG, "plan %d: image is NULL", i);
  }
  return WS_OK;
}

ws_status run_batch(ws_batch* b, const int64_t* m, const double* const* uvw,
                    const void* const* vis, const float* const* weight,
                    void* const* images) {
  return b->precision == WS_FP64
             ? batch_image_impl<double>(b, m, uvw, vis, weight, images)
             : batch_image_impl<float>(b, m, uvw, vis, weight, images);
}

// Fills a plan over the given buffers and enqueues its twiddle tables.
ws_status init_plan(ws_plan* pl, const ws_params* params, int64_t max_vis,
                    const Layout& L, int dev, void* planes, void* work,
                    void* hip_stream) {
  pl->p = *params;
  pl->max_vis = max_vis;
  pl->L = L;
  pl->g = make_geo(params, L);
  pl->planes = planes;
  pl->work = static_cast<unsigned char*>(work);
  pl->stream = static_cast<hipStream_t>(hip_stream);
  pl->state = kEmpty;
  pl->device = dev;
  pl->cus = 256;
  {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount,
                              dev) == hipSuccess && n > 0)
      pl->cus = n;
  }
  pl->profile = false;
  WS_TRY(launch(pl, "zero_line", [&] {
    launch_zero_u32(pl->w<uint32_t>(L.o_zero), 64, pl->stream);
  }));
  if (params->correct) {
    double* corr = pl->w<double>(L.o_corr);
    pl->g.corr = corr;
    WS_TRY(launch(pl, "correction",
                  [&] { launch_correction(pl->g, corr, pl->stream); }));
  }
  if (params->precision == WS_FP64) {
    return launch(pl, "twiddles", [&] {
      launch_twiddles<double>(pl->work + L.o_tw_u, params->nu, pl->stream);
      launch_twiddles<double>(pl->work + L.o_tw_v, params->nv, pl->stream);
    });
  }
  return launch(pl, "twiddles", [&] {
    launch_twiddles<float>(pl->work + L.o_tw_u, params->nu, pl->stream);
    launch_twiddles<float>(pl->work + L.o_tw_v, params->nv, pl->stream);
  });
}

// ---- allocation-free imaging ---------------------------------------------
// The plane stack and the workspace of ws_grid_image_noalloc live in this
// fixed device array (one copy per GPU the library runs on, held until the
// process ends).  Host code never passes `scratch` itself to a kernel: the
// name is a host-side stand-in, so the device address of each GPU's copy is
// looked up once per device with hipGetSymbolAddress and used instead.
constexpr size_t kNoAllocBytes = WS_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch (dev must be current).
ws_status scratch_of_device(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return fail(WS_UNSUPPORTED_SIZE, "device %d: at most %d devices", dev,
                kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return fail(WS_HIP_ERROR, "hipGetSymbolAddress(scratch) on device %d: "
                  "%s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return WS_OK;
}

}  // namespace

extern "C" {

ws_status ws_validate_params(const ws_params* params) {
  return check_params(params);
}

ws_status ws_workspace_bytes(const ws_params* params, int64_t max_vis,
                             size_t* planes_bytes, size_t* work_bytes) {
  Layout L;
  WS_TRY(make_layout(params, max_vis, &L));
  if (planes_bytes) *planes_bytes = L.planes_bytes;
  if (work_bytes) *work_bytes = L.total;
  return WS_OK;
}

ws_status ws_kernel_transform(const ws_params* params, int64_t n,
                              const double* f, double* psi, double* cnorm) {
  WS_TRY(check_params(params));
  if (n < 0 || (n > 0 && (f == nullptr || psi == nullptr)))
    return fail(WS_INVALID_ARG, "n=%lld with f or psi NULL", (long long)n);
  Layout L{};
  L.T = 16;
  const Geo g = make_geo(params, L);
  for (int64_t i = 0; i < n; ++i)
    psi[i] = kernel_transform(g.kern, g.K, g.inv2s2, g.es_beta, f[i]);
  if (cnorm != nullptr) *cnorm = g.cnorm;
  return WS_OK;
}

ws_status ws_grid_init(const ws_params* params, int64_t max_vis, void* planes,
                       size_t planes_bytes, void* work, size_t work_bytes,
                       void* hip_stream, ws_plan** out) {
  if (out == nullptr) return fail(WS_INVALID_ARG, "out is NULL");
  *out = nullptr;
  Layout L;
  WS_TRY(make_layout(params, max_vis, &L));
  if (planes == nullptr || work == nullptr)
    return fail(WS_INVALID_ARG, "planes or work is NULL");
  if (!aligned(planes, 256) || !aligned(work, 256))
    return fail(WS_INVALID_ARG, "planes and work must be 256-byte aligned");
  if (planes_bytes < L.planes_bytes)
    return fail(WS_WORKSPACE_TOO_SMALL, "planes: %zu bytes < %zu needed",
                planes_bytes, L.planes_bytes);
  if (work_bytes < L.total)
    return fail(WS_WORKSPACE_TOO_SMALL, "work: %zu bytes < %zu needed",
                work_bytes, L.total);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess)
    return fail(WS_HIP_ERROR, "hipGetDevice failed (no GPU?)");
  ws_plan* pl = new (std::nothrow) ws_plan();
  if (pl == nullptr) return fail(WS_INVALID_ARG, "out of host memory");
  const ws_status st = init_plan(pl, params, max_vis, L, dev, planes, work,
                                 hip_stream);
  if (st != WS_OK) {
    delete pl;
    return st;
  }
  *out = pl;
  return WS_OK;
}

ws_status ws_grid_visibilities(ws_plan* plan, int64_t m, const double* uvw,
                               const void* vis, const float* weight,
                               int64_t* n_dropped_taps) {
  WS_TRY(check_plan(plan));
  WS_TRY(check_vis_args(plan, m, uvw, weight));
  if (m > 0 && vis == nullptr) return fail(WS_INVALID_ARG, "vis is NULL");
  if (!aligned(vis, plan->L.elem) || !aligned(n_dropped_taps, 8))
    return fail(WS_INVALID_ARG, "misaligned vis or n_dropped_taps");
  if (plan->state == kTransformed)
    return fail(WS_BAD_STATE,
                "the stack holds transforms; call ws_plan_reset first");
  const VisSource src = flat_source(uvw, vis, weight);
  if (plan->p.precision == WS_FP64)
    return grid_impl<double>(plan, m, src, n_dropped_taps);
  return grid_impl<float>(plan, m, src, n_dropped_taps);
}

ws_status ws_fft_planes(ws_plan* plan, int32_t direction) {
  WS_TRY(check_plan(plan));
  if (direction != 1 && direction != -1)
    return fail(WS_INVALID_ARG, "direction=%d: use +1 or -1", direction);
  const bool f64 = plan->p.precision == WS_FP64;
  if (plan->state == kEmpty) {
    WS_TRY(f64 ? zero_planes<double>(plan) : zero_planes<float>(plan));
    plan->state = kTransformed;
    return WS_OK;
  }
  WS_TRY(f64 ? fft_impl<double>(plan, direction)
             : fft_impl<float>(plan, direction));
  plan->state = kTransformed;
  return WS_OK;
}

ws_status ws_wcorrect_accumulate(ws_plan* plan, void* image) {
  WS_TRY(check_plan(plan));
  if (image == nullptr) return fail(WS_INVALID_ARG, "image is NULL");
  if (!aligned(image, plan->L.elem))
    return fail(WS_INVALID_ARG, "misaligned image");
  if (plan->state == kEmpty) return WS_OK;  // all planes are zero
  if (plan->state != kTransformed)
    return fail(WS_BAD_STATE,
                "the stack holds gridded planes, not transforms; call "
                "ws_fft_planes first (or ws_image_accumulate)");
  return launch(plan, "wcorrect", [&] {
    if (plan->p.precision == WS_FP64)
      launch_wcorrect<double>(plan->planes, image, plan->g, plan->stream);
    else
      launch_wcorrect<float>(plan->planes, image, plan->g, plan->stream);
  });
}

ws_status ws_image_accumulate(ws_plan* plan, void* image) {
  WS_TRY(check_plan(plan));
  if (image == nullptr) return fail(WS_INVALID_ARG, "image is NULL");
  if (!aligned(image, plan->L.elem))
    return fail(WS_INVALID_ARG, "misaligned image");
  if (plan->state == kTransformed)
    return fail(WS_BAD_STATE,
                "the stack already holds transforms; use "
                "ws_wcorrect_accumulate");
  if (plan->state == kEmpty) return WS_OK;
  ws_status st = plan->p.precision == WS_FP64
                     ? image_impl<double>(plan, image)
                     : image_impl<float>(plan, image);
  plan->state = kEmpty;
  return st;
}

ws_status ws_grid_image(ws_plan* plan, int64_t m, const double* uvw,
                        const void* vis, const float* weight, void* image,
                        int64_t* n_dropped_taps) {
  WS_TRY(check_plan(plan));
  WS_TRY(check_vis_args(plan, m, uvw, weight));
  if (m > 0 && vis == nullptr) return fail(WS_INVALID_ARG, "vis is NULL");
  if (image == nullptr) return fail(WS_INVALID_ARG, "image is NULL");
  if (!aligned(vis, plan->L.elem) || !aligned(image, plan->L.elem) ||
      !aligned(n_dropped_taps, 8))
    return fail(WS_INVALID_ARG, "misaligned vis, image or n_dropped_taps");
  if (plan->state != kEmpty)
    return fail(WS_BAD_STATE,
                "the stack is not empty; call ws_plan_reset first");
  return grid_image_impl(plan, m, flat_source(uvw, vis, weight), image,
                         n_dropped_taps);
}

ws_status ws_grid_rows(ws_plan* plan, int64_t nrows, int32_t nchan,
                       int32_t npol, const double* uvw_m,
                       const double* freq_hz, const void* vis,
                       const float* weight, const double* pol_coeff,
                       int64_t* n_dropped_taps) {
  WS_TRY(check_plan(plan));
  VisSource src;
  int64_t m = 0;
  WS_TRY(rows_source(plan, nrows, nchan, npol, uvw_m, freq_hz, vis, weight,
                     pol_coeff, &src, &m));
  if (!aligned(n_dropped_taps, 8))
    return fail(WS_INVALID_ARG, "misaligned n_dropped_taps");
  if (plan->state == kTransformed)
    return fail(WS_BAD_STATE,
                "the stack holds transforms; call ws_plan_reset first");
  if (plan->p.precision == WS_FP64)
    return grid_impl<double>(plan, m, src, n_dropped_taps);
  return grid_impl<float>(plan, m, src, n_dropped_taps);
}

ws_status ws_grid_image_rows(ws_plan* plan, int64_t nrows, int32_t nchan,
                             int32_t npol, const double* uvw_m,
                             const double* freq_hz, const void* vis,
                             const float* weight, const double* pol_coeff,
                             void* image, int64_t* n_dropped_taps) {
  WS_TRY(check_plan(plan));
  VisSource src;
  int64_t m = 0;
  WS_TRY(rows_source(plan, nrows, nchan, npol, uvw_m, freq_hz, vis, weight,
                     pol_coeff, &src, &m));
  if (image == nullptr) return fail(WS_INVALID_ARG, "image is NULL");
  if (!aligned(image, plan->L.elem) || !aligned(n_dropped_taps, 8))
    return fail(WS_INVALID_ARG, "misaligned image or n_dropped_taps");
  if (plan->state != kEmpty)
    return fail(WS_BAD_STATE,
                "the stack is not empty; call ws_plan_reset first");
  return grid_image_impl(plan, m, src, image, n_dropped_taps);
}

ws_status ws_degrid(ws_plan* plan, const void* image, int32_t image_is_real,
                    int64_t m, const double* uvw, const float* weight,
                    void* vis_out) {
  WS_TRY(check_plan(plan));
  WS_TRY(check_vis_args(plan, m, uvw, weight));
  if (image == nullptr) return fail(WS_INVALID_ARG, "image is NULL");
  if (m > 0 && vis_out == nullptr)
    return fail(WS_INVALID_ARG, "vis_out is NULL");
  const size_t ea = image_is_real ? plan->L.elem / 2 : plan->L.elem;
  if (!aligned(image, ea) || !aligned(vis_out, plan->L.elem))
    return fail(WS_INVALID_ARG, "misaligned image or vis_out");
  ws_status st = plan->p.precision == WS_FP64
                     ? degrid_impl<double>(plan, image, image_is_real != 0, m,
                                           uvw, weight, vis_out)
                     : degrid_impl<float>(plan, image, image_is_real != 0, m,
                                          uvw, weight, vis_out);
  plan->state = kEmpty;
  return st;
}

ws_status ws_grid_image_noalloc(const ws_params* params, int64_t m,
                                const double* uvw, const void* vis,
                                const float* weight, void* image,
                                int64_t* n_dropped_taps, void* hip_stream) {
  // Sizes first (host only): a problem that does not fit the scratch is
  // refused before any device work.
  Layout L;
  WS_TRY(make_layout(params, m > 0 ? m : 1, &L));
  const size_t planes_at = 0;
  const size_t work_at = align_up(L.planes_bytes, 256);
  const size_t need = work_at + L.total;
  if (need > kNoAllocBytes)
    return fail(WS_WORKSPACE_TOO_SMALL,
                "this problem needs %zu bytes of stack and workspace; the "
                "allocation-free call has a %zu-byte static scratch (use "
                "ws_grid_init with caller buffers instead)",
                need, kNoAllocBytes);
  if (image == nullptr) return fail(WS_INVALID_ARG, "image is NULL");
  if (m > 0 && vis == nullptr) return fail(WS_INVALID_ARG, "vis is NULL");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess)
    return fail(WS_HIP_ERROR, "hipGetDevice failed (no GPU?)");
  unsigned char* base = nullptr;
  WS_TRY(scratch_of_device(dev, &base));
  ws_plan pl;  // host object on this stack frame: nothing is allocated
  WS_TRY(init_plan(&pl, params, m > 0 ? m : 1, L, dev, base + planes_at,
                   base + work_at, hip_stream));
  WS_TRY(check_vis_args(&pl, m, uvw, weight));
  if (!aligned(vis, L.elem) || !aligned(image, L.elem) ||
      !aligned(n_dropped_taps, 8))
    return fail(WS_INVALID_ARG, "misaligned vis, image or n_dropped_taps");
  return grid_image_impl(&pl, m, flat_source(uvw, vis, weight), image,
                         n_dropped_taps);
}

ws_status ws_dirty_beam(ws_plan* plan, int64_t m, const double* uvw,
                        const float* weight, void* image_scratch, void* beam,
                        double* beta) {
  WS_TRY(check_plan(plan));
  WS_TRY(check_vis_args(plan, m, uvw, weight));
  if (image_scratch == nullptr || beam == nullptr || beta == nullptr)
    return fail(WS_INVALID_ARG, "image_scratch, beam or beta is NULL");
  if (!aligned(image_scratch, plan->L.elem) ||
      !aligned(beam, plan->L.elem / 2) || !aligned(beta, 8))
    return fail(WS_INVALID_ARG, "misaligned image_scratch, beam or beta");
  if (plan->state != kEmpty)
    return fail(WS_BAD_STATE,
                "the stack is not empty; call ws_plan_reset first");
  const bool f64 = plan->p.precision == WS_FP64;
  const int64_t npix = (int64_t)plan->p.nu * plan->p.nv;
  WS_TRY(launch(plan, "fill_zero", [&] {
    if (f64) launch_fill_zero<double>(image_scratch, npix, plan->stream);
    else launch_fill_zero<float>(image_scratch, npix, plan->stream);
  }));
  WS_TRY(grid_image_impl(plan, m, flat_source(uvw, nullptr, weight),
                         image_scratch, nullptr));
  return launch(plan, "beam_normalise", [&] {
    if (f64)
      launch_beam_normalise<double>(image_scratch, beam, beta, plan->p.nu,
                                    plan->p.nv, plan->stream);
    else
      launch_beam_normalise<float>(image_scratch, beam, beta, plan->p.nu,
                                   plan->p.nv, plan->stream);
  });
}

ws_status ws_residual_image(ws_plan* plan, int64_t m, const double* uvw,
                            const void* vis, const float* weight,
                            const void* model, const double* beta,
                            void* vis_scratch, void* image_scratch,
                            void* residual) {
  WS_TRY(check_plan(plan));
  WS_TRY(check_vis_args(plan, m, uvw, weight));
  if (model == nullptr || beta == nullptr || image_scratch == nullptr ||
      residual == nullptr || (m > 0 && (vis == nullptr ||
                                        vis_scratch == nullptr)))
    return fail(WS_INVALID_ARG, "a buffer argument is NULL");
  const size_t e = plan->L.elem;
  if (!aligned(vis, e) || !aligned(vis_scratch, e) ||
      !aligned(image_scratch, e) || !aligned(model, e / 2) ||
      !aligned(residual, e / 2) || !aligned(beta, 8))
    return fail(WS_INVALID_ARG, "misaligned buffer argument");
  const bool f64 = plan->p.precision == WS_FP64;
  const int64_t npix = (int64_t)plan->p.nu * plan->p.nv;
  // Predicted visibilities of the model (unit weights), then R = V - pred.
  ws_status st = f64 ? degrid_impl<double>(plan, model, 1, m, uvw, nullptr,
                                           vis_scratch)
                     : degrid_impl<float>(plan, model, 1, m, uvw, nullptr,
                                          vis_scratch);
  plan->state = kEmpty;
  WS_TRY(st);
  WS_TRY(launch(plan, "residual_vis", [&] {
    if (f64) launch_residual_vis<double>(vis, vis_scratch, m, plan->stream);
    else launch_residual_vis<float>(vis, vis_scratch, m, plan->stream);
  }));
  WS_TRY(launch(plan, "fill_zero", [&] {
    if (f64) launch_fill_zero<double>(image_scratch, npix, plan->stream);
    else launch_fill_zero<float>(image_scratch, npix, plan->stream);
  }));
  WS_TRY(grid_image_impl(plan, m, flat_source(uvw, vis_scratch, weight),
                         image_scratch, nullptr));
  return launch(plan, "real_scale", [&] {
    if (f64)
      launch_real_scale<double>(image_scratch, residual, beta, npix,
                                plan->stream);
    else
      launch_real_scale<float>(image_scratch, residual, beta, npix,
                               plan->stream);
  });
}

ws_status ws_clean_minor(ws_plan* plan, void* residual, const void* beam,
                         void* model, int32_t niter, double gain,
                         double threshold, int32_t* picks, int32_t* n_done) {
  WS_TRY(check_plan(plan));
  if (residual == nullptr || beam == nullptr || model == nullptr)
    return fail(WS_INVALID_ARG, "residual, beam or model is NULL");
  if (niter < 0) return fail(WS_INVALID_ARG, "niter=%d < 0", niter);
  if (!(gain > 0.0 && gain <= 1.0))
    return fail(WS_INVALID_ARG, "gain must lie in (0, 1]");
  if (!(threshold >= 0.0) || !std::isfinite(threshold))
    return fail(WS_INVALID_ARG, "threshold must be finite and >= 0");
  const size_t e = plan->L.elem / 2;
  if (!aligned(residual, e) || !aligned(beam, e) || !aligned(model, e) ||
      !aligned(picks, 4) || !aligned(n_done, 4))
    return fail(WS_INVALID_ARG, "misaligned buffer argument");
  const int64_t npix = (int64_t)plan->p.nu * plan->p.nv;
  int64_t ns = (npix + 2047) / 2048;  // ~8 pixels per thread and block
  if (ns > kCleanMaxSlots) ns = kCleanMaxSlots;
  if (ns < 1) ns = 1;
  CleanState* state = plan->w<CleanState>(plan->L.o_clean);
  CleanSlot* slots = reinterpret_cast<CleanSlot*>(
      plan->work + plan->L.o_clean + sizeof(CleanState));
  return launch(plan, "clean_minor", [&] {
    if (plan->p.precision == WS_FP64)
      launch_clean_minor<double>(residual, beam, model, plan->p.nu,
                                 plan->p.nv, niter, gain, threshold, state,
                                 slots, (int)ns, picks, n_done,
                                 plan->stream);
    else
      launch_clean_minor<float>(residual, beam, model, plan->p.nu,
                                plan->p.nv, niter, gain, threshold, state,
                                slots, (int)ns, picks, n_done, plan->stream);
  });
}

ws_status ws_plan_reset(ws_plan* plan) {
  if (plan == nullptr) return fail(WS_INVALID_ARG, "plan is NULL");
  plan->state = kEmpty;
  return WS_OK;
}

ws_status ws_set_stream(ws_plan* plan, void* hip_stream) {
  if (plan == nullptr) return fail(WS_INVALID_ARG, "plan is NULL");
  plan->stream = static_cast<hipStream_t>(hip_stream);
  return WS_OK;
}

ws_status ws_sync(ws_plan* plan) {
  WS_TRY(check_plan(plan));
  const hipError_t e = hipStreamSynchronize(plan->stream);
  if (e != hipSuccess)
    return fail(WS_HIP_ERROR, "stream error: %s", hipGetErrorString(e));
  return WS_OK;
}

ws_status ws_tile_stats(ws_plan* plan, int64_t out[7]) {
  WS_TRY(check_plan(plan));
  if (out == nullptr) return fail(WS_INVALID_ARG, "out is NULL");
  uint32_t c[8];
  const size_t nstrips = (size_t)plan->g.nw * plan->g.tiles_u;
  std::vector<uint32_t> marks(nstrips);
  hipError_t e = hipStreamSynchronize(plan->stream);
  if (e == hipSuccess)
    e = hipMemcpy(c, plan->w<uint32_t>(plan->L.o_counters), sizeof(c),
                  hipMemcpyDeviceToHost);
  if (e == hipSuccess)
    e = hipMemcpy(marks.data(), plan->w<uint32_t>(plan->L.o_strips),
                  nstrips * sizeof(uint32_t), hipMemcpyDeviceToHost);
  if (e != hipSuccess)
    return fail(WS_HIP_ERROR, "reading the tile counts: %s",
                hipGetErrorString(e));
  int64_t marked = 0;
  for (uint32_t v : marks) marked += v != 0u;
  out[0] = plan->g.T;
  out[1] = c[4];
  out[2] = c[5];
  out[3] = c[1];
  out[4] = c[2];
  out[5] = marked;
  out[6] = (int64_t)((uint64_t)c[6] | ((uint64_t)c[7] << 32));
  return WS_OK;
}

ws_status ws_set_profiling(ws_plan* plan, int32_t enable) {
  if (plan == nullptr) return fail(WS_INVALID_ARG, "plan is NULL");
  plan->profile = enable != 0;
  return WS_OK;
}

ws_status ws_kernel_times(ws_plan* plan, int32_t cap, const char** names,
                          double* total_ms, int64_t* launches, int32_t* n,
                          int32_t reset) {
  WS_TRY(check_plan(plan));
  if (hipStreamSynchronize(plan->stream) != hipSuccess)
    return fail(WS_HIP_ERROR, "stream error while collecting times");
  for (auto& pe : plan->pending) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, pe.a, pe.b) == hipSuccess) {
      plan->ms[pe.id] += t;
      plan->launches[pe.id] += 1;
    }
    hipEventDestroy(pe.a);
    hipEventDestroy(pe.b);
  }
  plan->pending.clear();
  const int32_t cnt = (int32_t)plan->names.size();
  for (int32_t i = 0; i < cnt && i < cap; ++i) {
    if (names) names[i] = plan->names[i];
    if (total_ms) total_ms[i] = plan->ms[i];
    if (launches) launches[i] = plan->launches[i];
  }
  if (n) *n = cnt;
  if (reset) {
    for (auto& v : plan->ms) v = 0.0;
    for (auto& v : plan->launches) v = 0;
  }
  return WS_OK;
}

ws_status ws_batch_workspace_bytes(int32_t n, size_t* work_bytes) {
  if (n < 1 || n > kMaxBatch)
    return fail(WS_INVALID_ARG, "n=%d: a batch holds 1..%d plans", n,
                kMaxBatch);
  if (work_bytes) *work_bytes = batch_jobs_bytes(n) + 256;
  return WS_OK;
}

ws_status ws_batch_create(int32_t n, ws_plan* const* plans, void* work,
                          size_t work_bytes, ws_batch** out) {
  if (out == nullptr) return fail(WS_INVALID_ARG, "out is NULL");
  *out = nullptr;
  size_t need = 0;
  WS_TRY(ws_batch_workspace_bytes(n, &need));
  if (plans == nullptr || work == nullptr)
    return fail(WS_INVALID_ARG, "plans or work is NULL");
  if (work_bytes < need)
    return fail(WS_WORKSPACE_TOO_SMALL, "work: %zu bytes < %zu needed",
                work_bytes, need);
  if (!aligned(work, 256))
    return fail(WS_INVALID_ARG, "work must be 256-byte aligned");
  for (int i = 0; i < n; ++i) {
    if (plans[i] == nullptr) return fail(WS_INVALID_ARG, "plan %d is NULL", i);
    if (plans[i]->p.precision != plans[0]->p.precision ||
        plans[i]->p.support != plans[0]->p.support ||
        plans[i]->p.kernel != plans[0]->p.kernel ||
        plans[i]->device != plans[0]->device)
      return fail(WS_INVALID_ARG,
                  "plan %d: all plans of a batch share precision, support, "
                  "kernel type and device", i);
    for (int j2 = 0; j2 < i; ++j2)
      if (plans[j2] == plans[i])
        return fail(WS_INVALID_ARG, "plan %d appears twice", i);
  }
  WS_TRY(check_plan(plans[0]));
  ws_batch* b = new (std::nothrow) ws_batch();
  if (b == nullptr) return fail(WS_INVALID_ARG, "out of host memory");
  b->n = n;
  b->plans.assign(plans, plans + n);
  b->work = static_cast<unsigned char*>(work);
  b->precision = plans[0]->p.precision;
  b->K = plans[0]->p.support;
  b->kern = plans[0]->p.kernel;
  b->stream = plans[0]->stream;
  b->graph = nullptr;
  b->exec = nullptr;
  b->lds = 0;
  std::vector<unsigned char> host(batch_jobs_bytes(n), 0);
  for (int i = 0; i < n; ++i) {
    const size_t lds = grid_lds_bytes(plans[i]->L.T, b->K,
                                      b->precision == WS_FP64 ? 8 : 4);
    if (lds > b->lds) b->lds = lds;
    if (b->precision == WS_FP64) {
      const GridJob<double> j = make_job<double>(plans[i], 0);
      std::memcpy(host.data() + i * sizeof(GridJob<double>), &j, sizeof(j));
    } else {
      const GridJob<float> j = make_job<float>(plans[i], 0,
                                               tstore_ok(plans[i]));
      std::memcpy(host.data() + i * sizeof(GridJob<float>), &j, sizeof(j));
    }
  }
  if (hipMemcpy(b->work, host.data(), host.size(), hipMemcpyHostToDevice) !=
      hipSuccess) {
    delete b;
    return fail(WS_HIP_ERROR, "copying the batch job table failed");
  }
  *out = b;
  return WS_OK;
}

ws_status ws_batch_image(ws_batch* b, const int64_t* m,
                         const double* const* uvw, const void* const* vis,
                         const float* const* weight, void* const* images) {
  WS_TRY(check_batch_args(b, m, uvw, vis, images));
  WS_TRY(check_plan(b->plans[0]));
  return run_batch(b, m, uvw, vis, weight, images);
}

ws_status ws_batch_capture(ws_batch* b, const int64_t* m,
                           const double* const* uvw, const void* const* vis,
                           const float* const* weight, void* const* images) {
  WS_TRY(check_batch_args(b, m, uvw, vis, images));
  WS_TRY(check_plan(b->plans[0]));
  if (b->stream == nullptr)
    return fail(WS_BAD_STATE, "capture needs a non-null stream");
  if (b->exec != nullptr) {
    hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph != nullptr) {
    hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  std::vector<bool> prof(b->n);
  for (int i = 0; i < b->n; ++i) {
    prof[i] = b->plans[i]->profile;
    b->plans[i]->profile = false;  // no event records inside the graph
  }
  if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) !=
      hipSuccess)
    return fail(WS_HIP_ERROR, "hipStreamBeginCapture failed");
  ws_status st = run_batch(b, m, uvw, vis, weight, images);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->stream, &g);
  for (int i = 0; i < b->n; ++i) b->plans[i]->profile = prof[i];
  if (st != WS_OK) {
    if (g) hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess || g == nullptr)
    return fail(WS_HIP_ERROR, "hipStreamEndCapture failed: %s",
                hipGetErrorString(e));
  if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    hipGraphDestroy(g);
    b->exec = nullptr;
    return fail(WS_HIP_ERROR, "hipGraphInstantiate failed");
  }
  b->graph = g;
  return WS_OK;
}

ws_status ws_batch_replay(ws_batch* b) {
  if (b == nullptr) return fail(WS_INVALID_ARG, "batch is NULL");
  if (b->exec == nullptr)
    return fail(WS_BAD_STATE, "nothing captured: call ws_batch_capture");
  WS_TRY(check_plan(b->plans[0]));
  const hipError_t e = hipGraphLaunch(b->exec, b->stream);
  if (e != hipSuccess)
    return fail(WS_HIP_ERROR, "hipGraphLaunch failed: %s",
                hipGetErrorString(e));
  return WS_OK;
}

void ws_batch_destroy(ws_batch* b) {
  if (b == nullptr) return;
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  delete b;
}

void ws_plan_destroy(ws_plan* plan) {
  if (plan == nullptr) return;
  for (auto& pe : plan->pending) {
    hipEventDestroy(pe.a);
    hipEventDestroy(pe.b);
  }
  delete plan;
}

const char* ws_status_string(ws_status status) {
  switch (status) {
    case WS_OK: return "WS_OK";
    case WS_INVALID_ARG: return "WS_INVALID_ARG";
    case WS_UNSUPPORTED_SIZE: return "WS_UNSUPPORTED_SIZE";
    case WS_WORKSPACE_TOO_SMALL: return "WS_WORKSPACE_TOO_SMALL";
    case WS_HIP_ERROR: return "WS_HIP_ERROR";
    case WS_BAD_STATE: return "WS_BAD_STATE";
    default: return "WS_UNKNOWN_STATUS";
  }
}

const char* ws_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
