// Shared device-side definitions of the w-stacking library: complex types,
// the per-plan geometry block every kernel receives, the FP64 visibility
// placement (Sec. 2: nearest cell and nearest w-plane) and the bin-key
// layout used by the binning, gridding and degridding kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace ws {

template <typename R>
struct cplx {
  R re, im;
};

template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

template <typename R>
__device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) {
  return {a.re + b.re, a.im + b.im};
}

template <typename R>
__device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) {
  return {a.re - b.re, a.im - b.im};
}

// Number of bin regions per tile: a tile's cells split into a 3 x 3 pattern
// of edge strips (width h) and the interior, so that the records a
// neighbouring tile needs form a few contiguous key ranges.
constexpr int kRegions = 9;
constexpr uint32_t kNoKey = 0xFFFFFFFFu;
// Key counts are kept in kCountCopies copies: workgroup b of the counting
// kernel adds into copy b % kCountCopies, so the atomics on one key (the
// densely sampled centre of the uv plane puts many visibilities on a few
// keys) spread over that many addresses; the workgroups of one copy run on
// one XCD when blocks are dealt to the XCDs in turn.  The copies are then
// turned into per-copy offsets; any assignment of workgroups to copies
// gives the same records.
constexpr int kCountCopies = 8;
// Integer cell indices are packed into 16 bits each with this offset.
constexpr int kCellBias = 64;

// Geometry block passed by value to every kernel.
struct Geo {
  int nu, nv, nw;      // grid size and plane count
  int K, h;            // kernel support and half-width
  int T;               // gridding tile edge (cells)
  int tiles_u, tiles_v;
  int ntiles;          // nw * tiles_u * tiles_v
  double fov_l, fov_m; // full field of view (radians)
  double w_min, dw;    // plane origin and spacing (dw unused when nw == 1)
  double w0;           // centre of plane 0
  double dl, dm;       // pixel size in direction cosines
  double inv2s2;       // 1 / (2 sigma^2), FP64
  float kappa;         // log2(e) / (2 sigma^2), FP32 (exp2 form)
  double cnorm;        // kernel norm c: the 2-D kernel integrates to one
  // Exponential-of-semicircle kernel phi(d) = exp(beta (sqrt(1 - z^2) - 1)),
  // z = 2 d / K (used when kern == kKernelES).
  int kern;            // kKernelGauss or kKernelES
  double es_beta;      // beta
  double es_zs;        // 2 / K
  float es_beta2;      // beta log2(e) (FP32 exp2 form)
  float es_zs_f;       // 2 / K in FP32
  // Grid correction: null, or the device table of nu + nv FP64 factors
  // whose product corr[p] corr[nu + q] is 1 / (c psi(f_p) psi(f_q)).
  const double* corr;
  // Row order of a transformed stack: 0 = natural; otherwise the columns
  // went through a four-step transform of nv = perm_n1 * perm_n2 and row
  // k1 * perm_n2 + k2 holds column frequency k1 + perm_n1 * k2.
  int perm_n1, perm_n2;
};

// Gridding kernels (Sec. 2, the paragraph after Eq. 3: the paper's Gaussian,
// and the exponential of a semicircle as the analytic stand-in for the
// production kernels it names).
constexpr int kKernelGauss = 0;
constexpr int kKernelES = 1;

// psi(f) = integral over |d| <= K/2 of phi(d) cos(2 pi f d) dd: the Fourier
// transform of the truncated 1-D kernel at f cycles per cell, in FP64.
// Tanh-sinh (double-exponential) quadrature over the half interval
// [0, K/2] (the integrand is even): d = (K/4)(1 + tanh(s)),
// s = (pi/2) sinh(t), t = j h; its node density grows double-exponentially
// at both ends, which absorbs the square-root edge of the ES kernel.  The
// distance of a node from the far end, K/2 - d = (K/2) / (1 + e^(2s)), is
// formed directly so that 1 - z^2 = (1 - z)(1 + z) keeps full precision
// next to the edge.  h = 1/32 over |t| <= 3.2 (205 nodes) converges to
// FP64 rounding for every supported kernel.
__host__ __device__ inline double kernel_transform(int kern, int K,
                                                   double inv2s2, double beta,
                                                   double f) {
  const double a = 0.5 * (double)K;  // half-width of the support
  const double h = 1.0 / 32.0;
  const double pi = 3.14159265358979323846;
  double sum = 0.0;
  for (int j = -102; j <= 102; ++j) {
    const double t = (double)j * h;
    const double s = 0.5 * pi * sinh(t);
    const double e = exp(2.0 * s);
    const double far = a / (1.0 + e);     // K/2 - d
    const double d = a - far;
    const double ch = cosh(s);
    const double wt = h * 0.5 * a * (0.5 * pi * cosh(t)) / (ch * ch);
    double phi;
    if (kern == kKernelES) {
      const double omz = far / a;         // 1 - z
      const double z = 1.0 - omz;
      const double r = sqrt(omz * (1.0 + z) > 0.0 ? omz * (1.0 + z) : 0.0);
      phi = exp(-beta * z * z / (1.0 + r));
    } else {
      phi = exp(-inv2s2 * d * d);
    }
    sum += wt * phi * cos(2.0 * pi * f * d);
  }
  return 2.0 * sum;
}

// Row of the stack that holds column frequency q.
__host__ __device__ inline int stack_row(const Geo& g, int q) {
  return g.perm_n1 == 0 ? q : (q % g.perm_n1) * g.perm_n2 + q / g.perm_n1;
}

// Column frequency held by row r of the stack.
__host__ __device__ inline int stack_freq(const Geo& g, int r) {
  return g.perm_n1 == 0 ? r : r / g.perm_n2 + g.perm_n1 * (r % g.perm_n2);
}

// FP64 placement of one visibility.  Contraction is off so that the cell
// position and the plane index round exactly as the separate IEEE multiply,
// add and divide of the definition.  Returns false when every tap of the
// visibility falls off the grid (including non-finite coordinates).
__host__ __device__ inline bool place(const Geo& g, double u, double v,
                                      double w, double& x, double& y, int& i0,
                                      int& j0, int& k) {
#pragma clang fp contract(off)
  x = u * g.fov_l + 0.5 * (double)g.nu;
  y = v * g.fov_m + 0.5 * (double)g.nv;
  // x - x is 0 for every finite x and NaN for NaN and +-Inf.
  if (!(u - u == 0.0 && v - v == 0.0 && w - w == 0.0)) return false;
  if (!(fabs(x) < 1.0e9 && fabs(y) < 1.0e9)) return false;
  const double fi = floor(x + 0.5);
  const double fj = floor(y + 0.5);
  if (fi < -g.h || fi > g.nu - 1 + g.h || fj < -g.h || fj > g.nv - 1 + g.h)
    return false;
  i0 = (int)fi;
  j0 = (int)fj;
  if (g.nw == 1) {
    k = 0;
  } else {
    double t = floor((w - g.w_min) / g.dw);
    t = t < 0.0 ? 0.0 : t;
    t = t > (double)(g.nw - 1) ? (double)(g.nw - 1) : t;
    k = (int)t;
  }
  return true;
}

// Number of the K*K taps of a visibility centred on (i0, j0) that lie on
// the grid.
__host__ __device__ inline int taps_on_grid(const Geo& g, int i0, int j0) {
  int lo = i0 - g.h < 0 ? 0 : i0 - g.h;
  int hi = i0 + g.h > g.nu - 1 ? g.nu - 1 : i0 + g.h;
  const int cols = hi >= lo ? hi - lo + 1 : 0;
  lo = j0 - g.h < 0 ? 0 : j0 - g.h;
  hi = j0 + g.h > g.nv - 1 ? g.nv - 1 : j0 + g.h;
  const int rows = hi >= lo ? hi - lo + 1 : 0;
  return cols * rows;
}

// Region of a tile-local coordinate along one axis: 0 = the strip within h
// of the low edge, 2 = within h of the high edge, 1 = interior.
__host__ __device__ inline int strip(int local, int T, int h) {
  return local < h ? 0 : (local >= T - h ? 2 : 1);
}

// Regions are numbered around the tile's rim, then the interior:
//   (ry, rx): (0,0)=0 (0,1)=1 (0,2)=2 (1,2)=3 (2,2)=4 (2,1)=5 (2,0)=6 (1,0)=7
//   (1,1)=8.
// With this order, the records a neighbouring tile needs (one edge: three
// regions; one corner: one region) are a single key range, except the
// low-u edge, which is two.
__host__ __device__ inline int region_code(int ry, int rx) {
  // Selects rather than a table, which the device compiler would place in
  // memory and load per call.
  const int mid = rx == 0 ? 7 : (rx == 1 ? 8 : 3);
  return ry == 0 ? rx : (ry == 2 ? 6 - rx : mid);
}

// Bin key of a placed visibility: (plane, tile row, tile column, region).
// The home tile is the one holding the nearest cell, clamped to the grid.
__host__ __device__ inline uint32_t bin_key(const Geo& g, int i0, int j0,
                                            int k) {
  const int ic = i0 < 0 ? 0 : (i0 > g.nu - 1 ? g.nu - 1 : i0);
  const int jc = j0 < 0 ? 0 : (j0 > g.nv - 1 ? g.nv - 1 : j0);
  const int tx = ic / g.T, ty = jc / g.T;
  const int rx = strip(ic - tx * g.T, g.T, g.h);
  const int ry = strip(jc - ty * g.T, g.T, g.h);
  const uint32_t tile =
      ((uint32_t)k * (uint32_t)g.tiles_v + (uint32_t)ty) * (uint32_t)g.tiles_u +
      (uint32_t)tx;
  return tile * kRegions + (uint32_t)region_code(ry, rx);
}

// One binned visibility, stored whole (array of structures) so that the
// scatter of a visibility into its bin is one 24-byte (FP32) or 40-byte
// (FP64) write and the gridder reads a record with three 8-byte loads
// (FP32); no padding rides in the binning and gridding streams.
//   dx, dy  offset of the exact position from the nearest cell
//   vr, vi  weighted visibility (gridding) or weight and 0 (degridding)
//   cell    packed nearest cell (pack_cell)
//   idx     input index of the visibility (degridding)
template <typename R>
struct alignas(8) Record {
  R dx, dy, vr, vi;
  uint32_t cell, idx;
};
static_assert(sizeof(Record<float>) == 24 && sizeof(Record<double>) == 40,
              "records carry no padding");

__host__ __device__ inline uint32_t pack_cell(int i0, int j0) {
  return (uint32_t)(i0 + kCellBias) | ((uint32_t)(j0 + kCellBias) << 16);
}

__host__ __device__ inline int cell_i(uint32_t c) {
  return (int)(c & 0xFFFFu) - kCellBias;
}

__host__ __device__ inline int cell_j(uint32_t c) {
  return (int)(c >> 16) - kCellBias;
}

// The key ranges (in units of keys) of the records whose kernel footprint
// reaches tile t: its own nine regions plus the facing strips and corners
// of its up to eight neighbours.  Always writes kSegments [lo, hi) pairs in
// fixed slots (a missing neighbour leaves its slot empty, lo == hi), so
// that callers can keep them in registers.
constexpr int kSegments = 10;
__host__ __device__ inline void tile_segments(const Geo& g, int t,
                                              uint32_t lo[kSegments],
                                              uint32_t hi[kSegments]) {
  const int per_plane = g.tiles_u * g.tiles_v;
  const int k = t / per_plane;
  const int rem = t - k * per_plane;
  const int ty = rem / g.tiles_u;
  const int tx = rem - ty * g.tiles_u;
  const uint32_t base = (uint32_t)k * per_plane;
  auto key0 = [&](int yy, int xx) {
    return (base + (uint32_t)(yy * g.tiles_u + xx)) * kRegions;
  };
  const bool L = tx > 0, Rt = tx + 1 < g.tiles_u;
  const bool A = ty > 0, B = ty + 1 < g.tiles_v;
  // slot: (present, neighbour row, neighbour column, first region, end)
  auto put = [&](int s, bool on, int yy, int xx, uint32_t r0, uint32_t r1) {
    const uint32_t k0 = on ? key0(yy, xx) : 0u;
    lo[s] = on ? k0 + r0 : 0u;
    hi[s] = on ? k0 + r1 : 0u;
  };
  put(0, true, ty, tx, 0, 9);
  put(1, Rt, ty, tx + 1, 6, 8);   // right neighbour's low-u strip: 6, 7
  put(2, Rt, ty, tx + 1, 0, 1);   //   ... and 0
  put(3, L, ty, tx - 1, 2, 5);    // left neighbour's high-u strip
  put(4, B, ty + 1, tx, 0, 3);    // next row's low-v strip
  put(5, A, ty - 1, tx, 4, 7);    // previous row's high-v strip
  put(6, Rt && B, ty + 1, tx + 1, 0, 1);
  put(7, L && B, ty + 1, tx - 1, 2, 3);
  put(8, Rt && A, ty - 1, tx + 1, 6, 7);
  put(9, L && A, ty - 1, tx - 1, 4, 5);
}

}  // namespace ws
