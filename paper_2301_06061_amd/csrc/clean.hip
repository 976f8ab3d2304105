// Imaging major cycle: the kernels around the imaging path that a
// Cotton-Schwab deconvolution needs (Sec. 1: imaging is followed by CLEAN
// deconvolution, with Hogbom's image-plane loop and the major / minor
// split of Clark and Schwab).
//
//   k_beam_normalise   dirty beam = Re(image of unit visibilities) divided
//                      by its centre value beta (beta kept on the device)
//   k_residual_vis     R = V - predicted (in place over the prediction)
//   k_real_scale       residual image = Re(image) / beta
//   k_clean_step       Hogbom minor cycle, step t: subtract component t - 1
//                      (gain * peak times the beam centred on its pixel,
//                      truncated at the edges) and find each block's largest
//                      |D| in the same pass over the image
//   k_clean_pick       one workgroup: the winner among the blocks (ties: the
//                      lowest pixel index), the threshold test, the model
//                      update and the pending component for the next step
//
// The minor cycle runs as niter (step, pick) launch pairs plus one final
// step, with every decision kept in device memory: the host never waits
// inside the cycle.  A step reads the residual and the beam and writes the
// residual once (HBM-bound; the search rides along with the subtraction).
#include <type_traits>

#include "ws_kernels.h"

namespace ws {

namespace {

constexpr int kCleanThreads = 256;

// Argmax candidate: larger |v| wins; equal |v|: the lower index wins.
// Non-finite magnitudes never win (comparisons with NaN are false).
struct Cand {
  double mag;
  double val;
  int64_t idx;
};

__device__ __forceinline__ bool better(const Cand& a, const Cand& b) {
  return a.mag > b.mag || (a.mag == b.mag && a.idx < b.idx);
}

__device__ __forceinline__ Cand shfl_cand(const Cand& c, int src) {
  Cand o;
  o.mag = __shfl(c.mag, src, 64);
  o.val = __shfl(c.val, src, 64);
  o.idx = __shfl(c.idx, src, 64);
  return o;
}

// Largest candidate of the workgroup, valid in thread 0.
__device__ __forceinline__ Cand block_best(Cand c, Cand* s_c) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const Cand d = shfl_cand(c, (lane + o) & 63);
    if (lane + o < 64 && better(d, c)) c = d;
  }
  if (lane == 0) s_c[wave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
      if (better(s_c[w], c)) c = s_c[w];
  }
  return c;
}

template <typename R>
__global__ __launch_bounds__(256) void k_beam_normalise(
    const cplx<R>* __restrict__ img, R* __restrict__ beam,
    double* __restrict__ beta_out, int nu, int nv) {
  const double beta = (double)img[(size_t)(nv / 2) * nu + nu / 2].re;
  const int64_t n = (int64_t)nu * nv;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = i0; i < n; i += stride)
    beam[i] = (R)((double)img[i].re / beta);
  if (i0 == 0) *beta_out = beta;
}

template <typename R>
__global__ __launch_bounds__(256) void k_residual_vis(
    const cplx<R>* __restrict__ vis, cplx<R>* __restrict__ pred, int64_t m) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = i0; i < m; i += stride) pred[i] = csub(vis[i], pred[i]);
}

template <typename R>
__global__ __launch_bounds__(256) void k_real_scale(
    const cplx<R>* __restrict__ img, R* __restrict__ out,
    const double* __restrict__ beta, int64_t n) {
  const double b = *beta;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = i0; i < n; i += stride)
    out[i] = (R)((double)img[i].re / b);
}

// Subtract the pending component (if any) and find this block's largest
// |D|.  Pixels are taken V at a time (one 16-byte load of D when the
// buffers allow it, else V = 1) in a grid-stride loop, so the blocks cover
// the image evenly; the beam index of pixel (p, q) for a component at
// (p*, q*) is (q - q* + nv/2, p - p* + nu/2), skipped where it leaves the
// beam.  nu is a power of two (2^lognu), so a group of V pixels lies in
// one row.  Within a thread the pixels come in increasing index, so a
// strictly larger |D| is the only way to replace the candidate (ties keep
// the lower index); the comparisons run in the path precision, which
// orders |D| exactly as FP64 would.  `search` = 0 for the final
// subtraction after the last pick.
template <typename R, int V>
__global__ __launch_bounds__(kCleanThreads) void k_clean_step(
    R* __restrict__ d, const R* __restrict__ beam, int nu, int nv, int lognu,
    const CleanState* __restrict__ st, CleanSlot* __restrict__ slots,
    int search) {
  __shared__ Cand s_c[kCleanThreads / 64];
  using Vec = typename std::conditional<
      V == 1, R,
      typename std::conditional<sizeof(R) == 4, float4, double2>::type>::type;
  static_assert(V * sizeof(R) == sizeof(Vec), "V values per load");
  const int64_t n = (int64_t)nu * nv;
  const bool sub = st->pending != 0;
  const int64_t pidx = st->pend_idx;
  const int pq = (int)(pidx >> lognu), pp = (int)(pidx & (nu - 1));
  const R amp = (R)st->pend_amp;
  R bmag = (R)-1, bval = (R)0;
  int64_t bidx = n;
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * V;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * V;
  for (int64_t i = i0; i < n; i += stride) {
    Vec raw = *reinterpret_cast<const Vec*>(d + i);
    R* v = reinterpret_cast<R*>(&raw);
    if (sub) {
      const int q = (int)(i >> lognu), p = (int)(i & (nu - 1));
      const int bq = q - pq + nv / 2, bp = p - pp + nu / 2;
      if ((unsigned)bq < (unsigned)nv) {
        const R* brow = beam + (size_t)bq * nu;
        bool any = false;
#pragma unroll
        for (int j = 0; j < V; ++j) {
          if ((unsigned)(bp + j) < (unsigned)nu) {
            v[j] = v[j] - amp * brow[bp + j];
            any = true;
          }
        }
        if (any) *reinterpret_cast<Vec*>(d + i) = raw;
      }
    }
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const R m = fabs(v[j]);
      if (m > bmag) {
        bmag = m;
        bval = v[j];
        bidx = i + j;
      }
    }
  }
  if (!search) return;
  const Cand best = block_best(Cand{(double)bmag, (double)bval, bidx}, s_c);
  if (threadIdx.x == 0) {
    slots[blockIdx.x].mag = best.mag;
    slots[blockIdx.x].val = best.val;
    slots[blockIdx.x].idx = best.idx;
  }
}

// The winner of the blocks; stop on the threshold or after niter picks,
// else add gain * peak to the model and make it the pending component.
template <typename R>
__global__ __launch_bounds__(kCleanThreads) void k_clean_pick(
    const CleanSlot* __restrict__ slots, int nslots, CleanState* st,
    R* __restrict__ model, int32_t* __restrict__ picks, double gain,
    double threshold, int32_t* __restrict__ n_done) {
  __shared__ Cand s_c[kCleanThreads / 64];
  Cand best{-1.0, 0.0, INT64_MAX};
  for (int s = threadIdx.x; s < nslots; s += blockDim.x) {
    const Cand c{slots[s].mag, slots[s].val, slots[s].idx};
    if (better(c, best)) best = c;
  }
  best = block_best(best, s_c);
  if (threadIdx.x != 0) return;
  if (st->stopped || !(best.mag >= threshold) || best.mag < 0.0) {
    st->stopped = 1;
    st->pending = 0;
    return;
  }
  const double a = best.val;
  model[best.idx] = (R)((double)model[best.idx] + gain * a);
  if (picks != nullptr) picks[st->count] = (int32_t)best.idx;
  st->count += 1;
  if (n_done != nullptr) *n_done = st->count;
  st->pending = 1;
  st->pend_idx = best.idx;
  st->pend_amp = gain * a;
}

__global__ void k_clean_reset(CleanState* st, int32_t* n_done) {
  st->stopped = 0;
  st->pending = 0;
  st->count = 0;
  st->pend_idx = 0;
  st->pend_amp = 0.0;
  if (n_done != nullptr) *n_done = 0;
}

int grid_of(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

template <typename R>
void launch_beam_normalise(const void* img, void* beam, double* beta, int nu,
                           int nv, hipStream_t st) {
  hipLaunchKernelGGL(k_beam_normalise<R>, dim3(grid_of((int64_t)nu * nv)),
                     dim3(256), 0, st, (const cplx<R>*)img, (R*)beam, beta,
                     nu, nv);
}

template <typename R>
void launch_residual_vis(const void* vis, void* pred, int64_t m,
                         hipStream_t st) {
  if (m == 0) return;
  hipLaunchKernelGGL(k_residual_vis<R>, dim3(grid_of(m)), dim3(256), 0, st,
                     (const cplx<R>*)vis, (cplx<R>*)pred, m);
}

template <typename R>
void launch_real_scale(const void* img, void* out, const double* beta,
                       int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_real_scale<R>, dim3(grid_of(n)), dim3(256), 0, st,
                     (const cplx<R>*)img, (R*)out, beta, n);
}

template <typename R>
void launch_clean_minor(void* d, const void* beam, void* model, int nu,
                        int nv, int niter, double gain, double threshold,
                        CleanState* state, CleanSlot* slots, int nslots,
                        int32_t* picks, int32_t* n_done, hipStream_t st) {
  int lognu = 0;
  while ((1 << lognu) < nu) ++lognu;
  // 16-byte loads of the residual where it is 16-byte aligned (rows of a
  // power-of-two width keep every group of V pixels aligned then).
  constexpr int V = 16 / (int)sizeof(R);
  const bool vec = (reinterpret_cast<uintptr_t>(d) % 16) == 0 && nu % V == 0;
  hipLaunchKernelGGL(k_clean_reset, dim3(1), dim3(1), 0, st, state, n_done);
  for (int t = 0; t <= niter; ++t) {
    const int search = t < niter ? 1 : 0;
    if (vec)
      hipLaunchKernelGGL((k_clean_step<R, V>), dim3(nslots),
                         dim3(kCleanThreads), 0, st, (R*)d, (const R*)beam,
                         nu, nv, lognu, state, slots, search);
    else
      hipLaunchKernelGGL((k_clean_step<R, 1>), dim3(nslots),
                         dim3(kCleanThreads), 0, st, (R*)d, (const R*)beam,
                         nu, nv, lognu, state, slots, search);
    if (search)
      hipLaunchKernelGGL(k_clean_pick<R>, dim3(1), dim3(kCleanThreads), 0,
                         st, slots, nslots, state, (R*)model, picks, gain,
                         threshold, n_done);
  }
}

#define WS_INST(R)                                                            \
  template void launch_beam_normalise<R>(const void*, void*, double*, int,   \
                                         int, hipStream_t);                  \
  template void launch_residual_vis<R>(const void*, void*, int64_t,          \
                                       hipStream_t);                         \
  template void launch_real_scale<R>(const void*, void*, const double*,      \
                                     int64_t, hipStream_t);                  \
  template void launch_clean_minor<R>(void*, const void*, void*, int, int,   \
                                      int, double, double, CleanState*,      \
                                      CleanSlot*, int, int32_t*, int32_t*,   \
                                      hipStream_t);
WS_INST(float)
WS_INST(double)
#undef WS_INST

}  // namespace ws
