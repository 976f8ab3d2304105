// Host-side launchers of the w-stacking kernels (one translation unit per
// group: binning, gridding/degridding, FFT and screen).  Every launcher only
// enqueues work on the given stream; buffers are caller-owned device memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "ws_common.h"

namespace ws {

// Where the binning kernels read visibility i (0 <= i < m) from.
//   rows == 0 (flat): uvw[i] in wavelengths, vis[i], weight[i] (or unit);
//     the gridded value is weight[i] vis[i] (vis == null: unit
//     visibilities, the value is weight[i]).
//   rows == 1 (baseline-major, Sec. 2 data structures / Sec. 3.4.2 thread
//     loop): visibility i = r * nchan + c of row r (one baseline at one
//     time) and channel c; uvw[r] in metres, scaled by f_c / c0 to
//     wavelengths; vis[r][c][p] over npol correlations, weight[r][p] (or
//     unit); the gridded value is sum_p coef_p weight[r][p] vis[r][c][p]
//     (formed in FP64), e.g. a Stokes parameter from the correlations.
constexpr int kMaxPol = 4;
struct VisSource {
  const double* uvw;
  const void* vis;
  const float* weight;
  int rows;
  int nchan, npol;
  const double* freq;          // [nchan] Hz (rows only)
  double coef[kMaxPol][2];     // (re, im) per correlation (rows only)
};

// binning (bin.hip)
// Counts go to kCountCopies copies of nkeys words each (zeroed by the
// caller); fold them into totals, scan the totals, then turn the copies
// into per-copy offsets, which the scatter reads.
void launch_bin_count(const Geo& g, const VisSource& src, int64_t m,
                      uint32_t* copies, uint32_t nkeys, uint2* keyrank,
                      unsigned long long* dropped, hipStream_t st);
// Two-level partition (bin.hip): the same records and key offsets as the
// counting sort above, with no global atomics.  Buckets hold `span` keys
// each (a plane and a group of tile rows; nbuckets * span = all keys).
struct PartWork {
  uint32_t nbuckets, span;
  uint2* keyrank;      // [max_vis] key and rank in the workgroup's bucket
  uint32_t* hist1;     // [blocks][nbuckets] level-1 histograms, then
                       // the scanned (bucket, block) offsets in place
  uint32_t* hist1x;    // [blocks][nbuckets] each workgroup's exclusive scan
  uint32_t* btot;      // [blocks] records each workgroup placed
  uint32_t* bounds;    // [nbuckets + 1] first record of every bucket
  uint32_t* seg;       // [64][nbuckets] segment sums of the level-1 scan
  uint32_t* sums;      // scan scratch
  void* rec1;          // [max_vis] records in bucket order
  uint32_t* keys;      // [max_vis] their keys
  uint32_t* chunk0;    // [nbuckets + 1] first level-2 chunk of each bucket
  uint32_t* rank2;     // [max_vis] rank within (chunk, key)
  uint32_t* hist2;     // [chunks][span] level-2 histograms -> offsets
  uint32_t* hist2x;    // [chunks][span] each chunk's exclusive scan
  uint32_t* offsets;   // [nkeys + 1] record offset of every key
  void* rec;           // [max_vis] final records in key order
};
// Phases, in order: level-1 counts; the bucket-major scan and the
// level-2 chunks; the level-1 scatter; level-2 counts; level-2 scan (writes
// the key offsets); the level-2 scatter (writes the final records).
template <typename R>
void launch_part_count1(const Geo& g, const VisSource& src, int64_t m,
                        const PartWork& w, unsigned long long* dropped,
                        hipStream_t st);
template <typename R>
void launch_part_scan1(int64_t m, const PartWork& w, hipStream_t st);
template <typename R>
void launch_part_scatter1(const Geo& g, const VisSource& src, int64_t m,
                          const PartWork& w, int degrid, void* vis_out,
                          hipStream_t st);
template <typename R>
void launch_part_count2(int64_t m, const PartWork& w, hipStream_t st);
template <typename R>
void launch_part_scan2(int64_t m, const PartWork& w, hipStream_t st);
template <typename R>
void launch_part_scatter2(int64_t m, const PartWork& w, hipStream_t st);
// Workgroups of level 1 and chunks of level 2 for max_vis visibilities
// (elem: bytes of a complex value, 8 or 16).
int64_t partition_blocks(int64_t max_vis, int elem);
int64_t partition_chunks(int64_t max_vis, int64_t nbuckets, int elem);

void launch_fold_copies(const uint32_t* copies, uint32_t nkeys,
                        uint32_t* totals, hipStream_t st);
void launch_copy_offsets(uint32_t* copies, uint32_t nkeys,
                         const uint32_t* offsets, hipStream_t st);
int64_t scan_sums_len(int64_t n);
void launch_exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n,
                           uint32_t* sums, hipStream_t st);
template <typename R>
void launch_bin_scatter(const Geo& g, const VisSource& src, int64_t m,
                        const uint2* keyrank, const uint32_t* offsets,
                        uint32_t nkeys, void* records, int degrid,
                        void* vis_out, hipStream_t st);
// tslot (optional): busy-list index of every tile with records.
void launch_tile_work(const Geo& g, const uint32_t* offsets, int mode_degrid,
                      uint32_t chunk, uint32_t* tile_chunks,
                      uint32_t* tile_slot, uint32_t* counters,
                      uint32_t* split_list, uint32_t max_slots, uint2* extra,
                      uint32_t max_extra, uint32_t* busy, uint32_t* idle,
                      uint32_t* strips, uint32_t* tslot, hipStream_t st);

// gridding and degridding (grid.hip)
// LDS accumulator of the gridder: FP64 for both paths.  On gfx950 the
// LDS add of FP64 values (ds_add_f64) is far faster than that of FP32
// (the FP32 gridder measured 1.04 ms with FP64 sums and 5.1 ms with FP32
// sums on 1e7 visibilities), and FP64 sums keep the per-cell error of the
// FP32 path at the rounding of its inputs.
template <typename R>
struct GridAccOf {
  using type = double;
};
template <typename R>
using GridAcc = typename GridAccOf<R>::type;
int grid_lds_pitch(int T, int K);
// LDS bytes of one gridding tile (real and imaginary accumulators);
// real_bytes = 4 (FP32 path) or 8 (FP64).
size_t grid_lds_bytes(int T, int K, int real_bytes);
size_t degrid_lds_bytes(int T, int K, int elem_bytes);
// Everything one gridding launch needs for one plan (passed by value, or
// as an array in device memory for a batch).
constexpr int kMaxBatch = 64;
template <typename R>
struct GridJob {
  Geo g;
  int pitch;                  // LDS row pitch of the tile (FP64 words)
  const uint32_t* offsets;    // record offset of every key (+ total)
  uint32_t* counters;         // [1] split tiles, [2] extra items, [3] queue,
                              // [4] busy tiles, [5] idle tiles
  const uint2* extra;         // (tile, chunk) of the further chunks
  const uint32_t* busy;       // tiles with records ([4] of them)
  const uint32_t* idle;       // tiles without ([5]), zeroed separately
  const uint32_t* tile_chunks;
  const uint32_t* tile_slot;
  const Record<R>* rec;
  const uint32_t* desc;       // item descriptors (kDescWords words each)
  uint32_t chunk;
  cplx<R>* planes;
  cplx<R>* partials;
  int accumulate;
  int zero_idle;              // batch: this job's idle tiles need zeros
  // Busy-tile store (one-call path of 4096-row FP32 stacks): finished
  // tiles go to tstore[tslot[tile]] in column sub-blocks (tile_store_at)
  // instead of the stack; null = the stack.  Tiles whose busy-list index
  // (= slot) is tcap or more do not fit and go to the stack.
  cplx<R>* tstore;
  const uint32_t* tslot;
  uint32_t tcap;
};

// Element (row, col) of a tile of edge T in the busy-tile store: column
// sub-blocks of 64 bytes (8 FP32 columns) x T rows, one after another, so
// a column transform of 8 columns reads 512 contiguous bytes per tile row.
template <typename R>
__host__ __device__ inline size_t tile_store_at(int T, int row, int col) {
  constexpr int B = 64 / (int)sizeof(cplx<R>);
  return (size_t)(col / B) * T * B + (size_t)row * B + (col % B);
}

// Descriptors of the gridding work items (after launch_tile_work), one
// per item in queue order; desc holds max_items * kDescWords words.
constexpr int kDescWords = 24;
void launch_item_desc(const Geo& g, const uint32_t* offsets,
                      const uint32_t* counters, const uint2* extra,
                      const uint32_t* busy, const uint32_t* tile_chunks,
                      uint32_t chunk, uint32_t* desc, uint32_t max_items,
                      hipStream_t st);
template <typename R>
void launch_grid_tiles(const GridJob<R>& j, uint32_t max_items, int cus,
                       hipStream_t st);
template <typename R>
void launch_grid_batch(const GridJob<R>* jobs, int njobs, int K, int kern,
                       size_t lds, uint32_t* queue, uint32_t max_items,
                       int cus, hipStream_t st);
template <typename R>
void launch_zero_idle(const Geo& g, const uint32_t* counters,
                      const uint32_t* idle, void* planes, hipStream_t st);
template <typename R>
void launch_zero_idle_batch(const GridJob<R>* jobs, int njobs,
                            uint64_t total_tiles, hipStream_t st);
// With tstore (and tslot), merged tiles with a slot below tcap go to the
// busy-tile store.
template <typename R>
void launch_grid_merge(const Geo& g, const uint32_t* counters,
                       const uint32_t* split_list, const uint32_t* tile_chunks,
                       const uint32_t* tile_slot, const void* partials,
                       void* planes, int accumulate, uint32_t max_split,
                       void* tstore, const uint32_t* tslot, uint32_t tcap,
                       hipStream_t st);
template <typename R>
void launch_degrid_tiles(const Geo& g, const uint32_t* offsets,
                         uint32_t* counters, const uint2* extra,
                         const uint32_t* busy, const void* planes,
                         const void* records, uint32_t chunk,
                         void* vis_out, uint32_t max_items, int cus,
                         hipStream_t st);

// FFT and screen (fft.hip)
bool fft_supported(int n, int elem_bytes);
// Rows too long for two half-length LDS transforms take a 4-way split
// that writes through a scratch area of this many bytes (0 otherwise).
size_t fft_row_scratch_bytes(int n, int elem_bytes);
// Row transforms of nrows rows of n points.  With `strips` (marks of the
// 64-column strips of each plane of rows_per_plane rows), samples of
// unmarked strips are taken as zero and not read; false where the row
// kernel for n cannot (fft_rows_can_mask).
template <typename R>
bool launch_fft_rows(void* data, int n, int64_t nrows, const void* tw,
                     int sign, void* scratch, const uint32_t* strips,
                     int rows_per_plane, hipStream_t st);
bool fft_rows_can_mask(int n, int elem_bytes);
// Column transforms; with `strips` non-null, the blocks of column strips
// (strip_w columns of one plane) whose mark is zero are skipped; with
// `tiles` non-null (per-tile record counts, tile edge strip_w), rows of
// tiles without records are taken as zero and not read.  With `tstore`
// non-null (FP32, 4096 rows, strip_w 64, strips and tiles given) the
// tiles with records and a slot tslot[t] below tcap are read from the
// busy-tile store instead of `data`; false where that is not possible.
template <typename R>
bool launch_fft_cols(void* data, int nrows, int ncols, int nplanes,
                     const void* tw, int sign, const uint32_t* strips,
                     int strip_w, const uint32_t* tiles, const void* tstore,
                     const uint32_t* tslot, uint32_t tcap, hipStream_t st);
template <typename R>
bool launch_row_screen_sum(const void* planes, void* img, const Geo& g,
                           const void* tw_u, const uint32_t* strips,
                           hipStream_t st);
template <typename R>
bool launch_screen_row_bcast(const void* img, int img_real, void* planes,
                             const Geo& g, const void* tw_u, hipStream_t st);
// Four-step column transform (columns longer than 4096); with `tiles`
// (per-tile record counts, tile edge strip_w = 64, strips given), rows of
// tiles without records are taken as zero and not read (their loads go to
// `zeros`, 16 bytes of zeros in device memory).
template <typename R>
bool launch_fft_cols4(void* data, int nrows, int ncols, int nplanes,
                      const void* tw, int sign, const uint32_t* strips,
                      int strip_w, const uint32_t* tiles, const void* zeros,
                      hipStream_t st);
template <typename R>
void launch_unpermute_rows(const void* src, void* dst, const Geo& g,
                           hipStream_t st);
template <typename R>
void launch_screen_bcast(const void* img, int img_real, void* planes,
                         const Geo& g, hipStream_t st);
template <typename R>
void launch_wcorrect(const void* F, void* img, const Geo& g, hipStream_t st);
template <typename R>
void launch_fill_zero(void* p, int64_t n, hipStream_t st);
void launch_zero_u32(uint32_t* p, int64_t n, hipStream_t st);
template <typename R>
void launch_twiddles(void* tw, int n, hipStream_t st);
// Imaging major cycle (clean.hip).  Device state of one Hogbom minor
// cycle and the per-block argmax slots it reduces.
struct CleanState {
  int32_t stopped;    // threshold reached (or nothing finite to take)
  int32_t pending;    // a component awaits subtraction
  int32_t count;      // components taken
  int32_t pad;
  int64_t pend_idx;   // its pixel, q * nu + p
  double pend_amp;    // gain * peak
};
struct CleanSlot {
  double mag, val;
  int64_t idx;
};
constexpr int kCleanMaxSlots = 1024;
template <typename R>
void launch_beam_normalise(const void* img, void* beam, double* beta, int nu,
                           int nv, hipStream_t st);
template <typename R>
void launch_residual_vis(const void* vis, void* pred, int64_t m,
                         hipStream_t st);
template <typename R>
void launch_real_scale(const void* img, void* out, const double* beta,
                       int64_t n, hipStream_t st);
template <typename R>
void launch_clean_minor(void* d, const void* beam, void* model, int nu,
                        int nv, int niter, double gain, double threshold,
                        CleanState* state, CleanSlot* slots, int nslots,
                        int32_t* picks, int32_t* n_done, hipStream_t st);

// Grid-correction table of a plan (g.corr must point at nu + nv doubles):
// corr[p] = 1 / (c psi(f_p)), corr[nu + q] = 1 / psi(f_q), f = (index -
// n/2) / n, psi the kernel's 1-D transform (kernel_transform).
void launch_correction(const Geo& g, double* corr, hipStream_t st);

}  // namespace ws
