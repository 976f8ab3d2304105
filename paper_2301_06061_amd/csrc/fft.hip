// Batched 2-D FFT of the w-planes (Eq. 2, inner integral) and the fused
// w-screen kernels (Eq. 2, outer integral).
//
// Each 1-D transform is a Stockham autosort FFT (radix 8, one radix-4 or
// radix-2 stage last) held in LDS: the first stage reads HBM directly and
// the last writes HBM directly, so a transform costs one read and one write
// of its line.  Rows are transformed one per workgroup; columns in blocks of
// BC adjacent columns per workgroup (BC * 8 or 16 bytes per row segment),
// with the blocks that share a cache line placed on one XCD so that the
// partial lines are merged in that XCD's L2.  The centring
// (DC at N/2 in both domains) is a (-1)^index sign on input and output,
// valid for every N divisible by 4.  Twiddles e^{2 pi i t/N} come from
// tables computed in FP64 once per plan.
//
// Fused kernels: after the column stage, one workgroup per image row q
// transforms row q of every plane in turn and accumulates
// F_k[q][p] exp(2 pi i w_k (n_pq - 1)) in registers, so the transformed
// planes are never written back; the degridding counterpart multiplies an
// image row by each plane's conjugate screen before transforming it.  The
// screen phasor is advanced plane to plane by an FP64 complex multiply
// (the planes are equispaced in w), seeded with FP64 sincospi of the
// phase reduced to [-1/2, 1/2] turn.
#include "ws_kernels.h"

namespace ws {

namespace {

__device__ __forceinline__ uint32_t uniform_u32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

template <typename R>
__device__ __forceinline__ cplx<R> rot_i(cplx<R> a, R s) {
  // a * (s i)
  return {-s * a.im, s * a.re};
}

template <typename R>
__device__ __forceinline__ void dft2(cplx<R>* v) {
  const cplx<R> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <typename R>
__device__ __forceinline__ void dft4(cplx<R>* v, R s) {
  const cplx<R> a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
  const cplx<R> a2 = cadd(v[1], v[3]);
  const cplx<R> a3 = rot_i(csub(v[1], v[3]), s);
  v[0] = cadd(a0, a2);
  v[2] = csub(a0, a2);
  v[1] = cadd(a1, a3);
  v[3] = csub(a1, a3);
}

template <typename R>
__device__ __forceinline__ void dft8(cplx<R>* v, R s) {
  // Two length-4 transforms of the even and odd samples, then one radix-2
  // stage with the eighth roots of unity e^{s 2 pi i t/8}.
  cplx<R> e[4] = {v[0], v[2], v[4], v[6]};
  cplx<R> o[4] = {v[1], v[3], v[5], v[7]};
  dft4(e, s);
  dft4(o, s);
  const R h = (R)0.70710678118654752440084436210484903928;
  const cplx<R> o1 = {h * (o[1].re - s * o[1].im), h * (o[1].im + s * o[1].re)};
  const cplx<R> o2 = rot_i(o[2], s);
  const cplx<R> o3 = {h * (-o[3].re - s * o[3].im), h * (s * o[3].re - o[3].im)};
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

template <typename R, int RAD>
__device__ __forceinline__ void dft(cplx<R>* v, R s) {
  if constexpr (RAD == 8) dft8(v, s);
  else if constexpr (RAD == 4) dft4(v, s);
  else dft2(v);
}

// Twiddles e^{s 2 pi i idx/N} from two small LDS tables, e^{2 pi i lo/N}
// for lo < 64 and e^{2 pi i 64 hi/N}, both rounded from FP64 values.
template <typename R>
struct Twiddles {
  static constexpr bool kTable = false;
  const cplx<R>* t_lo;
  const cplx<R>* t_hi;
  __device__ __forceinline__ cplx<R> operator()(int idx, R s) const {
    const cplx<R> a = t_lo[idx & 63], b = t_hi[idx >> 6];
    const cplx<R> w = cmul(a, b);
    return {w.re, s * w.im};
  }
};

constexpr int kTwLo = 64;

// Fill the LDS twiddle tables of a length-n transform from the global table.
template <typename R>
__device__ __forceinline__ Twiddles<R> load_twiddles(cplx<R>* s_lo,
                                                     cplx<R>* s_hi,
                                                     const cplx<R>* tw, int n) {
  for (int i = threadIdx.x; i < kTwLo; i += blockDim.x) s_lo[i] = tw[i % n];
  for (int i = threadIdx.x; i < (n + kTwLo - 1) / kTwLo; i += blockDim.x)
    s_hi[i] = tw[i * kTwLo];
  return Twiddles<R>{s_lo, s_hi};
}

// Tables of a length-n sub-transform inside a length-nfull table
// (W_n^x = W_nfull^(x * nfull / n)), for the two steps of a four-step
// transform.
template <typename R>
__device__ __forceinline__ Twiddles<R> load_twiddles_sub(cplx<R>* s_lo,
                                                         cplx<R>* s_hi,
                                                         const cplx<R>* tw,
                                                         int n, int nfull) {
  const int stride = nfull / n;
  for (int i = threadIdx.x; i < kTwLo; i += blockDim.x)
    s_lo[i] = tw[((i % n) * stride) & (nfull - 1)];
  for (int i = threadIdx.x; i < (n + kTwLo - 1) / kTwLo; i += blockDim.x)
    s_hi[i] = tw[(i * kTwLo * stride) & (nfull - 1)];
  return Twiddles<R>{s_lo, s_hi};
}

// LDS slot of line element e: one padding slot after every 32 elements,
// so that the strided accesses of the Stockham stages spread over the
// banks (measured against one slot per 8, 16 and 64 elements: the fewest
// bank conflicts and the fastest column and row passes).
__device__ __forceinline__ constexpr int lslot(int e) { return e + (e >> 5); }

template <int N>
constexpr int lds_line(int bc) {
  return (N + (N + 31) / 32) * bc;
}

// Pass structure of a length-2^LOGN transform: radix 8, the remainder
// (radix 2 or 4) last; NS = product of the earlier radices.
constexpr int stage_npass(int logn) { return logn / 3 + (logn % 3 ? 1 : 0); }
constexpr int stage_rad(int logn, int P) {
  return P < logn / 3 ? 8 : (logn % 3 == 1 ? 2 : 4);
}
constexpr int stage_ns(int logn, int P) { return 1 << (3 * P); }
// Offset of stage P's entries in a stage twiddle table (stages 1 ..).
constexpr int stage_tw_off(int logn, int P) {
  int o = 0;
  for (int q = 1; q < P; ++q)
    o += (stage_rad(logn, q) - 1) * stage_ns(logn, q);
  return o;
}
constexpr int stage_tw_total(int logn) {
  return stage_tw_off(logn, stage_npass(logn));
}

// Twiddles of every stage held whole in LDS: stage P keeps
// W^(r k N / (NS RAD)) for r = 1 .. RAD-1, k < NS at
// tab[stage_tw_off(P) + (r - 1) NS + k] (lanes read consecutive k), the
// transform sign applied when the table is filled.  One LDS read per
// twiddle instead of a lookup and the powers of W^k: fewer vector
// instructions for kernels that transform many lines per table fill.
template <typename R>
struct TableTwiddles {
  static constexpr bool kTable = true;
  const cplx<R>* tab;
};

// Fills the stage table of a length-2^LOGN transform from the line's
// global table tw (W_N^i, i < N), conjugated for s = -1.  With
// `centred_in`, the last stage's entries also carry (-1)^r: a (-1)^e input
// centring gives every butterfly of the earlier stages one common sign,
// which the radix-8 Stockham order carries to input r of the last stage
// as (-1)^r, so the input needs no sign flips of its own.
template <typename R, int LOGN>
__device__ __forceinline__ void fill_stage_twiddles(cplx<R>* tab,
                                                    const cplx<R>* tw, R s,
                                                    bool centred_in) {
  constexpr int N = 1 << LOGN;
  constexpr int NPASS = stage_npass(LOGN);
  for (int i = threadIdx.x; i < stage_tw_total(LOGN); i += blockDim.x) {
    int idx = 0;
    bool neg = false;
#pragma unroll
    for (int P = 1; P < NPASS; ++P) {
      const int off = stage_tw_off(LOGN, P), ns = stage_ns(LOGN, P);
      const int rad = stage_rad(LOGN, P);
      if (i >= off && i < off + (rad - 1) * ns) {
        const int r = (i - off) / ns + 1, k = (i - off) % ns;
        idx = (r * k * (N / (ns * rad))) & (N - 1);
        neg = centred_in && P == NPASS - 1 && (r & 1);
      }
    }
    const cplx<R> w = tw[idx];
    tab[i] = neg ? cplx<R>{-w.re, -s * w.im} : cplx<R>{w.re, s * w.im};
  }
}

// Stage P of a length-2^LOGN Stockham FFT over BC interleaved columns
// (element e of column c at lds[e * BC + c]).  Stage 0 reads through
// ld(e, c); the last stage hands each output to st(e, c, it, r, value).
template <typename R, int LOGN, int BC, int NT, int P>
struct Stage {
  static constexpr int N = 1 << LOGN;
  static constexpr int NP8 = LOGN / 3;
  static constexpr int REM = LOGN % 3;
  static constexpr int NPASS = NP8 + (REM ? 1 : 0);
  static constexpr int RAD = P < NP8 ? 8 : (REM == 1 ? 2 : 4);
  static constexpr int NS = 1 << (3 * P);
  static constexpr int NB = N / RAD;
  static constexpr int TPC = NT / BC;
  static constexpr int IT = (NB + TPC - 1) / TPC;
  static constexpr bool FIRST = P == 0;
  static constexpr bool LAST = P == NPASS - 1;

  template <class Load, class Store, class TW>
  __device__ __forceinline__ static void run(cplx<R>* lds, const Load& ld,
                                             const Store& st, const TW& tw,
                                             R s) {
    const int c = threadIdx.x % BC;
    const int jt = threadIdx.x / BC;
    cplx<R> v[IT][RAD];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int j = jt + it * TPC;
      if (NB % TPC == 0 || j < NB) {
#pragma unroll
        for (int r = 0; r < RAD; ++r) {
          const int e = j + r * NB;
          if constexpr (FIRST) v[it][r] = ld(e, c, it, r);
          else v[it][r] = lds[lslot(e) * BC + c];
        }
      }
    }
    if constexpr (!FIRST) __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int j = jt + it * TPC;
      if (NB % TPC == 0 || j < NB) {
        const int k = j & (NS - 1);
        if constexpr (NS > 1 && TW::kTable) {
          constexpr int OFF = stage_tw_off(LOGN, P);
#pragma unroll
          for (int r = 1; r < RAD; ++r)
            v[it][r] = cmul(v[it][r], tw.tab[OFF + (r - 1) * NS + k]);
        } else if constexpr (NS > 1) {
          // Twiddles W^(r k N / (NS RAD)), r = 1 .. RAD-1, as powers of the
          // r = 1 value (one table lookup per butterfly; at most three
          // products deep, a few units in the last place).
          cplx<R> w[RAD];
          w[1] = tw(k * (N / (NS * RAD)), s);
          if constexpr (RAD > 2) {
            w[2] = cmul(w[1], w[1]);
            w[3] = cmul(w[2], w[1]);
          }
          if constexpr (RAD > 4) {
            w[4] = cmul(w[2], w[2]);
            w[5] = cmul(w[4], w[1]);
            w[6] = cmul(w[4], w[2]);
            w[7] = cmul(w[4], w[3]);
          }
#pragma unroll
          for (int r = 1; r < RAD; ++r) v[it][r] = cmul(v[it][r], w[r]);
        }
        dft<R, RAD>(v[it], s);
        if constexpr (LAST) {
#pragma unroll
          for (int r = 0; r < RAD; ++r) st(j + r * NB, c, it, r, v[it][r]);
        } else {
          const int ob = (j / NS) * NS * RAD + k;
#pragma unroll
          for (int r = 0; r < RAD; ++r)
            lds[lslot(ob + r * NS) * BC + c] = v[it][r];
        }
      }
    }
    if constexpr (!LAST) {
      __syncthreads();
      Stage<R, LOGN, BC, NT, P + 1>::run(lds, ld, st, tw, s);
    }
  }
};

template <typename R, int LOGN, int BC, int NT, class Load, class Store,
          class TW>
__device__ __forceinline__ void fft_line(cplx<R>* lds, const Load& ld,
                                         const Store& st, const TW& tw, R s) {
  Stage<R, LOGN, BC, NT, 0>::run(lds, ld, st, tw, s);
}

template <typename R>
__device__ __forceinline__ cplx<R> checker(cplx<R> v, int e) {
  return (e & 1) ? cplx<R>{-v.re, -v.im} : v;
}

// ---- plain row and column transforms (in place, any plane count) --------

// Sample e of a stack row whose 64-column strips carry marks (mk: the
// plane's marks, null when every strip holds data): read where the strip
// is marked, zero elsewhere (the load then goes to the spare line, so it
// costs no HBM traffic and needs no branch).  e - threadIdx.x must be the
// same across the workgroup and a multiple of 64, as in the first-stage
// loads of the row transforms, so that a wavefront's 64 samples lie in one
// strip and every choice here is wavefront-uniform.
template <bool MK, typename R>
__device__ __forceinline__ cplx<R> row_sample(const cplx<R>* line, int e,
                                              const uint32_t* __restrict__ mk,
                                              const cplx<R>* spare) {
  if constexpr (!MK) return line[e];
  const int c = e - (int)threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const bool on = mk[w + (c >> 6)] != 0u;
  const char* sb = on ? reinterpret_cast<const char*>(line + c)
                      : reinterpret_cast<const char*>(spare);
  const cplx<R> v = *reinterpret_cast<const cplx<R>*>(
      sb + (size_t)threadIdx.x * sizeof(cplx<R>));
  return cplx<R>{on ? v.re : (R)0, on ? v.im : (R)0};
}

// Marks of the plane that stack row `row` belongs to (null: no marks).
__device__ __forceinline__ const uint32_t* row_marks(const uint32_t* strips,
                                                     int64_t row,
                                                     int rows_per_plane,
                                                     int strips_per_row) {
  return strips == nullptr
             ? nullptr
             : strips + (size_t)(row / rows_per_plane) * strips_per_row;
}

// MK: with `strips` (marks of the 64-column strips of each plane of
// rows_per_plane rows), samples of unmarked strips are taken as zero and
// not read: the one-call path leaves those strips unwritten.
template <typename R, int LOGN, int NT, bool MK>
__global__ __launch_bounds__(NT) void k_fft_rows(
    cplx<R>* data, int64_t nrows, const cplx<R>* __restrict__ tw, R s,
    const uint32_t* __restrict__ strips, int rows_per_plane,
    int strips_per_row) {
  constexpr int N = 1 << LOGN;
  __shared__ cplx<R> lds[lds_line<N>(1)];
  __shared__ cplx<R> s_lo[kTwLo], s_hi[(N + kTwLo - 1) / kTwLo];
  const int64_t row = blockIdx.x;
  if (row >= nrows) return;
  const Twiddles<R> twl = load_twiddles(s_lo, s_hi, tw, N);
  __syncthreads();
  cplx<R>* line = data + row * N;
  static_assert(!MK || (NT % 64 == 0 && (N / 8) % 64 == 0),
                "marks need one strip per wavefront");
  const uint32_t* mk =
      MK ? row_marks(strips, row, rows_per_plane, strips_per_row) : nullptr;
  auto ld = [&](int e, int, int, int) {
    return checker(row_sample<MK>(line, e, mk, tw), e);
  };
  auto st = [&](int e, int, int, int, cplx<R> v) { line[e] = checker(v, e); };
  fft_line<R, LOGN, 1, NT>(lds, ld, st, twl, s);
}

template <typename R>
__device__ __forceinline__ cplx<R> twiddle_full(const cplx<R>* tw, int idx,
                                                R s) {
  const cplx<R> w = tw[idx];
  return {w.re, s * w.im};
}

// Rows too long for one workgroup's LDS (2N elements of FP64 at N = 16384):
// one radix-2 decimation-in-frequency step in registers, then two LDS
// transforms of half length.  With x' = (-1)^n x (centring),
//   X[2k]   = DFT_{N/2}( x'[n] + x'[n + N/2] )
//   X[2k+1] = DFT_{N/2}( (x'[n] - x'[n + N/2]) W_N^n ).
// Both halves of the row are read once (coalesced); the difference terms
// wait in registers while the sum terms are transformed, and the two
// outputs of each k are written together.
template <typename R, int LOGH, int NT, bool MK>
__global__ __launch_bounds__(NT) void k_fft_rows_split(
    cplx<R>* data, int64_t nrows, const cplx<R>* __restrict__ tw, R s,
    const uint32_t* __restrict__ strips, int rows_per_plane,
    int strips_per_row) {
  constexpr int NH = 1 << LOGH;  // half length
  constexpr int N = 2 * NH;
  __shared__ cplx<R> lds[lds_line<NH>(1)];
  __shared__ cplx<R> s_lo[kTwLo], s_hi[(NH + kTwLo - 1) / kTwLo];
  using F0 = Stage<R, LOGH, 1, NT, 0>;
  using FL = Stage<R, LOGH, 1, NT, F0::NPASS - 1>;
  const int64_t row = blockIdx.x;
  if (row >= nrows) return;
  cplx<R>* line = data + row * N;
  const Twiddles<R> twl = load_twiddles_sub(s_lo, s_hi, tw, NH, N);
  __syncthreads();
  cplx<R> diff[F0::IT][F0::RAD];
  cplx<R> even[FL::IT][FL::RAD];
  static_assert(!MK || (NT % 64 == 0 && F0::NB % 64 == 0 && NH % 64 == 0),
                "marks need one strip per wavefront");
  const uint32_t* mk =
      MK ? row_marks(strips, row, rows_per_plane, strips_per_row) : nullptr;
  auto ld_sum = [&](int e, int, int it, int r) {
    const cplx<R> a = checker(row_sample<MK>(line, e, mk, tw), e);
    const cplx<R> b = checker(row_sample<MK>(line, e + NH, mk, tw), e + NH);
    diff[it][r] = cmul(csub(a, b), twiddle_full(tw, e, s));
    return cadd(a, b);
  };
  auto st_even = [&](int, int, int it, int r, cplx<R> v) { even[it][r] = v; };
  fft_line<R, LOGH, 1, NT>(lds, ld_sum, st_even, twl, s);
  auto ld_diff = [&](int, int, int it, int r) { return diff[it][r]; };
  auto st_odd = [&](int e, int, int it, int r, cplx<R> v) {
    // output 2e is even (sign +1), 2e + 1 is odd (sign -1)
    const cplx<R> lo = even[it][r];
    const cplx<R> hi = {-v.re, -v.im};
    line[2 * e] = lo;
    line[2 * e + 1] = hi;
  };
  fft_line<R, LOGH, 1, NT>(lds, ld_diff, st_odd, twl, s);
}

// Rows too long even for two half-length LDS transforms (FP64 at 32768):
// F-way decimation in frequency with F = 4.  With x' = (-1)^n x and
// NF = N / F,
//   X[F k + r] = DFT_NF( W_N^(s r n) sum_m x'[n + m NF] W_F^(s m r) )[k],
// so output class r is one length-NF transform of a combination of the F
// samples x'[n + m NF]; output F k + r carries the centring sign (-1)^r.
// Pass r re-reads the row (F samples per point) instead of keeping the
// other classes in registers (at FP64 they would need ~200 registers a
// thread), and writes its outputs to the workgroup's row of `scratch`
// (every class reads the whole row, so nothing can be written in place
// before the last class); the finished row is then copied back.
// Persistent: workgroup b transforms rows b, b + G, ... (G = grid size),
// with scratch rows [G][N].  Only for grids wider than the fused kernels
// handle.
template <typename R, int LOGF, int NT, int F>
__global__ __launch_bounds__(NT) void k_fft_rows_splitF(
    cplx<R>* data, int64_t nrows, const cplx<R>* __restrict__ tw, R s,
    cplx<R>* __restrict__ scratch) {
  constexpr int NF = 1 << LOGF;
  constexpr int N = F * NF;
  __shared__ cplx<R> lds[lds_line<NF>(1)];
  __shared__ cplx<R> s_lo[kTwLo], s_hi[(NF + kTwLo - 1) / kTwLo];
  const Twiddles<R> twl = load_twiddles_sub(s_lo, s_hi, tw, NF, N);
  __syncthreads();
  cplx<R>* tmp = scratch + (size_t)blockIdx.x * N;
  for (int64_t row = blockIdx.x; row < nrows; row += gridDim.x) {
    cplx<R>* line = data + row * N;
    for (int r = 0; r < F; ++r) {
      auto ld = [&](int e, int, int, int) {
        cplx<R> acc = {(R)0, (R)0};
#pragma unroll
        for (int m = 0; m < F; ++m) {
          const int idx = e + m * NF;
          const cplx<R> x = checker(line[idx], idx);
          acc = cadd(acc,
                     cmul(x, twiddle_full(tw, (m * r * NF) & (N - 1), s)));
        }
        return cmul(acc, twiddle_full(tw, (r * e) & (N - 1), s));
      };
      const R sg = (r & 1) ? (R)-1 : (R)1;
      auto st = [&](int e, int, int, int, cplx<R> v) {
        tmp[F * e + r] = cplx<R>{sg * v.re, sg * v.im};
      };
      fft_line<R, LOGF, 1, NT>(lds, ld, st, twl, s);
      __syncthreads();
    }
    // Scratch row complete (global writes of this workgroup, ordered by
    // the barrier's release / acquire at workgroup scope): copy it back.
    __threadfence_block();
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += NT) line[i] = tmp[i];
    __syncthreads();
  }
}

// Workgroups of k_fft_rows_splitF (and scratch rows it needs).
constexpr int kSplitRowGroups = 256;

// Which rows of a column block hold data, from the per-tile record
// counts of gridding (0 = a tile without records, whose cells a fused
// grid-and-image call leaves unwritten and the transform takes as zero).
// The counts of the block's tile column (at most 64 tile rows) become one
// 64-bit mask per wavefront in the prologue, so every element then costs a
// shift and a select: no load, no branch, and the data loads of a
// wavefront still issue back to back.  Without a table every row holds
// data.
struct TileRows {
  unsigned long long mask;
  int log_t;
  // Issues the load of this lane's tile count (without a table, of any
  // valid word `any`, then ignored: the load stays unconditional and
  // nothing waits for it here); finish() turns the counts into the mask,
  // so other loads can be issued in between.
  __device__ __forceinline__ TileRows(const uint32_t* tiles, int plane,
                                      int nrows, int ncols, int col0,
                                      int log_t_, const void* any)
      : mask(~0ull), log_t(log_t_), rows(nrows >> log_t_),
        table(tiles != nullptr) {
    const int tw = ncols >> log_t;
    const int lane = (int)(threadIdx.x & 63);
    const uint32_t* src =
        table ? tiles + (size_t)plane * rows * tw + (col0 >> log_t) +
                    (size_t)min(lane, rows - 1) * tw
              : (const uint32_t*)any;
    count = *src;
  }
  __device__ __forceinline__ void finish() {
    const unsigned long long m =
        __ballot((int)(threadIdx.x & 63) < rows && count != 0u);
    mask = table ? m : ~0ull;
  }
  __device__ __forceinline__ bool has(int e) const {
    return ((mask >> (e >> log_t)) & 1ull) != 0ull;
  }
  // Sample of row e: loaded from p where the row holds data; elsewhere the
  // load goes to `spare` (one line that every such lane shares, so it costs
  // no HBM traffic) and the value is replaced by zero.  The load itself is
  // unconditional, so a wavefront issues its loads back to back.
  template <typename R>
  __device__ __forceinline__ cplx<R> load(int e, const cplx<R>* p,
                                          const cplx<R>* spare) const {
    const bool h = has(e);
    const cplx<R> v = *(h ? p : spare);
    return cplx<R>{h ? v.re : (R)0, h ? v.im : (R)0};
  }

 private:
  uint32_t count;
  int rows;
  bool table;
};

// Logical column block of hardware block b.  Blocks are dispatched to the
// eight XCDs in turn (b % 8); the G logical blocks that share one 128-byte
// line of every row are given to one XCD (they then share its L2), and
// successive groups go to successive XCDs, so every XCD holds an equal
// share of every plane (planes can differ widely in how many of their
// column strips are skipped).  Grids that are not a multiple of 8 G blocks
// keep the identity order.
template <typename R, int BC>
__device__ __forceinline__ int xcd_block(int b, int nb) {
  constexpr int W = BC * (int)sizeof(cplx<R>);
  constexpr int G = W >= 128 ? 1 : 128 / W;
  if (nb % (8 * G) != 0) return b;
  const int x = b % 8, n = b / 8;
  return ((n / G) * 8 + x) * G + n % G;
}

template <typename R, int LOGN, int BC, int NT>
__global__ __launch_bounds__(NT) void k_fft_cols(
    cplx<R>* data, int ncols, int nplanes, const cplx<R>* __restrict__ tw, R s,
    const uint32_t* __restrict__ strips, int log_strip,
    const uint32_t* __restrict__ tiles) {
  constexpr int N = 1 << LOGN;  // column length = number of rows
  __shared__ cplx<R> lds[lds_line<N>(BC)];
  __shared__ cplx<R> s_lo[kTwLo], s_hi[(N + kTwLo - 1) / kTwLo];
  const int nb_plane = ncols / BC;
  const int nb = nb_plane * nplanes;
  const int L = xcd_block<R, BC>((int)blockIdx.x, nb);
  if (L >= nb) return;
  const int plane = L / nb_plane;
  const int col0 = (L - plane * nb_plane) * BC;
  if (strips != nullptr &&
      strips[plane * (ncols >> log_strip) + (col0 >> log_strip)] == 0u)
    return;
  cplx<R>* base = data + (size_t)plane * N * ncols + col0;
  TileRows tr(tiles, plane, N, ncols, col0, log_strip, base);
  tr.finish();
  auto ld = [&](int e, int c, int, int) {
    return checker(tr.load(e, base + (size_t)e * ncols + c, tw), e);
  };
  auto st = [&](int e, int c, int, int, cplx<R> v) {
    base[(size_t)e * ncols + c] = checker(v, e);
  };
  const Twiddles<R> twl = load_twiddles(s_lo, s_hi, tw, N);
  __syncthreads();
  fft_line<R, LOGN, BC, NT>(lds, ld, st, twl, s);
}

// Column transform with twice the columns per workgroup that a whole
// column of LDS allows: one radix-2 decimation-in-frequency step as the
// samples arrive from HBM (rows e and e + N/2), the sums transformed in
// LDS first (outputs 2e, written at once: every input has been read)
// while the twiddled differences wait in registers, then the differences
// (outputs 2e + 1).  The wider block doubles the row segment each access
// moves (64 bytes instead of 32 for 4096-point FP32 columns).
//
// TS: the input tiles are read from the busy-tile store (tstore, slot of
// tile t at tslot[t], layout tile_store_at) instead of the stack: the BC
// columns of a block are one 64-byte sub-block of each tile, so every
// tile row a wavefront reads is 512 contiguous bytes.  Tiles with a slot
// of tcap or more did not fit the store and are read from the stack.
// Needs 64-row tiles and strips, BC = 64 bytes of columns and 64 rows per
// wavefront pass (TPC = 64); the output still goes to the stack.
template <typename R, int LOGH, int BC, int NT, bool TS>
__global__ __launch_bounds__(NT) void k_fft_cols_split(
    cplx<R>* data, int ncols, int nplanes, const cplx<R>* __restrict__ tw, R s,
    const uint32_t* __restrict__ strips, int log_strip,
    const uint32_t* __restrict__ tiles, const cplx<R>* __restrict__ tstore,
    const uint32_t* __restrict__ tslot, uint32_t tcap) {
  constexpr int NH = 1 << LOGH;  // half the column length
  constexpr int N = 2 * NH;
  __shared__ cplx<R> lds[lds_line<NH>(BC)];
  __shared__ cplx<R> s_lo[kTwLo], s_hi[(NH + kTwLo - 1) / kTwLo];
  __shared__ cplx<R> f_lo[kTwLo], f_hi[N / kTwLo];
  using F0 = Stage<R, LOGH, BC, NT, 0>;
  const int nb_plane = ncols / BC;
  const int nb = nb_plane * nplanes;
  const int L = xcd_block<R, BC>((int)blockIdx.x, nb);
  if (L >= nb) return;
  const int plane = L / nb_plane;
  const int col0 = (L - plane * nb_plane) * BC;
  if (strips != nullptr &&
      strips[plane * (ncols >> log_strip) + (col0 >> log_strip)] == 0u)
    return;
  cplx<R>* base = data + (size_t)plane * N * ncols + col0;
  // The loads of the prologue go first (the hardware returns loads in
  // order): one entry of the four twiddle tables per thread (W_NH^m and
  // W_NH^(64 m) for the half-length stages, W_N^m and W_N^(64 m) for the
  // difference terms), and the tile counts.
  static_assert(NT >= 4 * kTwLo && N / kTwLo <= kTwLo, "one entry a thread");
  const int tq = min((int)threadIdx.x / kTwLo, 3), tm = threadIdx.x % kTwLo;
  const int tidx = tq == 0   ? 2 * tm
                   : tq == 1 ? tm
                   : tq == 2 ? 2 * kTwLo * min(tm, NH / kTwLo - 1)
                             : kTwLo * min(tm, N / kTwLo - 1);
  const cplx<R> tval = tw[tidx];
  TileRows tr(tiles, plane, N, ncols, col0, log_strip, base);
  // TS: lane l holds the store slot of tile row l of this strip (any
  // value where the tile has no records: such rows are never read).
  int myslot = 0;
  if constexpr (TS) {
    const int rows = N >> log_strip, tcols = ncols >> log_strip;
    const int lane = (int)(threadIdx.x & 63);
    myslot = (int)tslot[((size_t)plane * rows + min(lane, rows - 1)) * tcols +
                        (col0 >> log_strip)];
  }
  if (threadIdx.x < 4 * kTwLo) {
    if (tq == 0) s_lo[tm] = tval;
    else if (tq == 1) f_lo[tm] = tval;
    else if (tq == 2) { if (tm < NH / kTwLo) s_hi[tm] = tval; }
    else if (tm < N / kTwLo) f_hi[tm] = tval;
  }
  tr.finish();
  const Twiddles<R> twl{s_lo, s_hi}, twf{f_lo, f_hi};
  __syncthreads();
  cplx<R> diff[F0::IT][F0::RAD];
  // The first stage takes the thread's sample pairs in order n = it * RAD +
  // r; the pair n + AHEAD is requested when pair n is combined, so each
  // wavefront keeps 2 AHEAD + 2 loads in flight without holding the whole
  // strip in registers (with one workgroup per CU there is no other
  // workgroup to hide the latency).  FP32 (512 threads, 256 registers)
  // runs 4 pairs ahead from the stack and 8 from the busy-tile store;
  // FP64 at 1024 threads has no registers to spare and loads each pair
  // where it is used (measured fastest for each; requesting every pair
  // before any arithmetic measured slower for both; from the store, 2, 4,
  // 6, 12 and 16 pairs ahead measured slower than 8).
  constexpr int AHEAD = sizeof(R) == 4 ? (TS ? 8 : 4) : 0;
  constexpr int NE = F0::IT * F0::RAD;
  const int c0 = (int)threadIdx.x % BC, jt = (int)threadIdx.x / BC;
  cplx<R> qa[NE], qb[NE];
  // TS addressing: row e = jt + it TPC + r NB lies in tile row
  // (it TPC + r NB) / 64 (a constant once unrolled; jt < 64) at row jt of
  // the tile, and the block's columns are sub-block (col0 % 64) / BC.  A
  // load address is a wavefront-uniform base (the tile's slot, the row
  // in the stack for a tile past the store's last slot, or the spare line
  // for a tile without records) plus one of two per-lane byte offsets, so
  // choosing between the three costs one vector select.
  const char* ts_base = nullptr;
  uint32_t v_ts = 0, v_st = 0;
  if constexpr (TS) {
    static_assert(F0::TPC == 64 && F0::NB % 64 == 0 && NH % 64 == 0 &&
                      BC * sizeof(cplx<R>) == 64,
                  "busy-tile store: 64-row tiles, 64-byte sub-blocks");
    ts_base = reinterpret_cast<const char*>(tstore) +
              (size_t)((col0 & 63) / BC) * (64 * BC) * sizeof(cplx<R>);
    v_ts = (uint32_t)((jt * BC + c0) * sizeof(cplx<R>));
    v_st = (uint32_t)(((size_t)jt * ncols + c0) * sizeof(cplx<R>));
  }
  // Row jt of tile row `trow` (a constant) whose store slot is s; every
  // choice below is wavefront-uniform.
  auto ts_load = [&](int trow, uint32_t s) {
    const bool h = ((tr.mask >> trow) & 1ull) != 0ull;
    const bool in = s < tcap;
    const char* sb =
        !h ? reinterpret_cast<const char*>(tw)
           : in ? ts_base + (size_t)s * (64 * 64 * sizeof(cplx<R>))
                : reinterpret_cast<const char*>(base) +
                      (size_t)trow * 64 * ncols * sizeof(cplx<R>);
    const cplx<R> v =
        *reinterpret_cast<const cplx<R>*>(sb + (size_t)(h && !in ? v_st : v_ts));
    return cplx<R>{h ? v.re : (R)0, h ? v.im : (R)0};
  };
  auto issue = [&](int n) {
    const int j = jt + (n / F0::RAD) * F0::TPC;
    if (F0::NB % F0::TPC == 0 || j < F0::NB) {
      const int e = j + (n % F0::RAD) * F0::NB;
      if constexpr (TS) {
        const int ta = ((n / F0::RAD) * F0::TPC + (n % F0::RAD) * F0::NB) / 64;
        qa[n] = ts_load(ta, __builtin_amdgcn_readlane(myslot, ta));
        qb[n] = ts_load(ta + NH / 64,
                        __builtin_amdgcn_readlane(myslot, ta + NH / 64));
      } else {
        qa[n] = tr.load(e, base + (size_t)e * ncols + c0, tw);
        qb[n] = tr.load(e + NH, base + (size_t)(e + NH) * ncols + c0, tw);
      }
    }
  };
#pragma unroll
  for (int n = 0; n < AHEAD && n < NE; ++n) issue(n);
  auto ld_sum = [&](int e, int, int it, int r) {
    const int n = it * F0::RAD + r;
    if (n + AHEAD < NE) issue(n + AHEAD);
    const cplx<R> a = checker(qa[n], e);
    const cplx<R> b = checker(qb[n], e + NH);
    diff[it][r] = cmul(csub(a, b), twf(e, s));
    return cadd(a, b);
  };
  // Output 2e has the centring sign +1, output 2e + 1 the sign -1.
  auto st_even = [&](int e, int c, int, int, cplx<R> v) {
    base[(size_t)(2 * e) * ncols + c] = v;
  };
  fft_line<R, LOGH, BC, NT>(lds, ld_sum, st_even, twl, s);
  auto ld_diff = [&](int, int, int it, int r) { return diff[it][r]; };
  auto st_odd = [&](int e, int c, int, int, cplx<R> v) {
    base[(size_t)(2 * e + 1) * ncols + c] = cplx<R>{-v.re, -v.im};
  };
  fft_line<R, LOGH, BC, NT>(lds, ld_diff, st_odd, twl, s);
}

// ---- four-step column transform for long columns (N = N1 * N2) ---------
//
// Step A: for each n2, the length-N1 transform over rows n1*N2 + n2, times
// W_N^(n2 k1), written back to row k1*N2 + n2.  Step B: for each k1, the
// length-N2 transform over the contiguous rows k1*N2 + n2; output k2 is
// frequency q = k1 + N1 k2 and is written back in place to row k1*N2 + k2.
// Each step reads and writes the stack once with 16-column (128- or
// 256-byte) row segments; the result has its rows in the transposed order
// that stack_row() undoes.

// TM: rows of tiles without records (tile counts `tiles`, tile edge
// strip_w = 64) are not read: their loads go to `zeros`, a line of zeros
// (the one-call path leaves those tiles unwritten).  Choosing the address,
// not the loaded value, keeps the loads free of branches.
template <typename R, int LOG1, int LOG2, int BC, int NT, bool TM>
__global__ __launch_bounds__(NT) void k_fft_colA(
    cplx<R>* data, int ncols, int nplanes, const cplx<R>* __restrict__ tw, R s,
    const uint32_t* __restrict__ strips, int strip_w,
    const uint32_t* __restrict__ tiles, const cplx<R>* __restrict__ zeros) {
  constexpr int N1 = 1 << LOG1, N2 = 1 << LOG2, N = N1 * N2;
  __shared__ cplx<R> lds[lds_line<N1>(BC)];
  __shared__ cplx<R> s_lo[kTwLo], s_hi[(N1 + kTwLo - 1) / kTwLo];
  __shared__ uint32_t s_tm[TM ? N / 64 : 1];
  const int ncb = ncols / BC;
  const int nb = ncb * N2 * nplanes;
  const int L = xcd_block<R, BC>((int)blockIdx.x, nb);
  if (L >= nb) return;
  const int cb = L % ncb;
  const int rest = L / ncb;
  const int n2 = rest % N2;
  const int plane = rest / N2;
  if (strips != nullptr &&
      strips[plane * (ncols / strip_w) + cb * BC / strip_w] == 0u)
    return;
  cplx<R>* base = data + (size_t)plane * N * ncols + (size_t)cb * BC;
  if constexpr (TM) {
    // Record counts of the strip's tiles, one per 64 rows.
    const int tcols = ncols / 64, strip = cb * BC / 64;
    for (int i = (int)threadIdx.x; i < N / 64; i += NT)
      s_tm[i] = tiles[((size_t)plane * (N / 64) + i) * tcols + strip];
  }
  const Twiddles<R> twl = load_twiddles_sub(s_lo, s_hi, tw, N1, N);
  __syncthreads();
  auto ld = [&](int e, int c, int, int) {
    const int row = e * N2 + n2;
    if constexpr (TM) {
      const bool h = s_tm[row >> 6] != 0u;
      return checker(*(h ? base + (size_t)row * ncols + c : zeros), row);
    } else {
      return checker(base[(size_t)row * ncols + c], row);
    }
  };
  auto st = [&](int e, int c, int, int, cplx<R> v) {
    const int row = e * N2 + n2;
    base[(size_t)row * ncols + c] =
        cmul(v, twiddle_full(tw, (n2 * e) & (N - 1), s));
  };
  fft_line<R, LOG1, BC, NT>(lds, ld, st, twl, s);
}

template <typename R, int LOG1, int LOG2, int BC, int NT>
__global__ __launch_bounds__(NT) void k_fft_colB(
    cplx<R>* data, int ncols, int nplanes, const cplx<R>* __restrict__ tw, R s,
    const uint32_t* __restrict__ strips, int strip_w) {
  constexpr int N1 = 1 << LOG1, N2 = 1 << LOG2, N = N1 * N2;
  __shared__ cplx<R> lds[lds_line<N2>(BC)];
  __shared__ cplx<R> s_lo[kTwLo], s_hi[(N2 + kTwLo - 1) / kTwLo];
  const int ncb = ncols / BC;
  const int nb = ncb * N1 * nplanes;
  const int L = xcd_block<R, BC>((int)blockIdx.x, nb);
  if (L >= nb) return;
  const int cb = L % ncb;
  const int rest = L / ncb;
  const int k1 = rest % N1;
  const int plane = rest / N1;
  if (strips != nullptr &&
      strips[plane * (ncols / strip_w) + cb * BC / strip_w] == 0u)
    return;
  cplx<R>* base = data + (size_t)plane * N * ncols + (size_t)k1 * N2 * ncols +
                  (size_t)cb * BC;
  const Twiddles<R> twl = load_twiddles_sub(s_lo, s_hi, tw, N2, N);
  __syncthreads();
  auto ld = [&](int e, int c, int, int) { return base[(size_t)e * ncols + c]; };
  auto st = [&](int e, int c, int, int, cplx<R> v) {
    base[(size_t)e * ncols + c] = checker(v, k1 + N1 * e);
  };
  fft_line<R, LOG2, BC, NT>(lds, ld, st, twl, s);
}

// Undo the transposed row order of a four-step column transform: copy row
// r of the plane to row q(r) of the scratch plane.
template <typename R>
__global__ __launch_bounds__(256) void k_unpermute_rows(
    const cplx<R>* __restrict__ src, cplx<R>* __restrict__ dst, Geo g) {
  const int r = blockIdx.y;
  const int q = stack_freq(g, r);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.nu;
       i += gridDim.x * blockDim.x)
    dst[(size_t)q * g.nu + i] = src[(size_t)r * g.nu + i];
}

// ---- w-screen -------------------------------------------------------------

// exp(2 pi i a) for a phase a in turns, reduced to [-1/2, 1/2] in FP64.
__device__ __forceinline__ cplx<double> turns_phasor(double a) {
  const double f = a - rint(a);
  double sn, cs;
  sincospi(2.0 * f, &sn, &cs);
  return {cs, sn};
}

// n - 1 = sqrt(1 - l^2 - m^2) - 1 in the cancellation-free form.
__device__ __forceinline__ double n_minus_one(const Geo& g, int p, int q) {
  const double l = (double)(p - g.nu / 2) * g.dl;
  const double m = (double)(q - g.nv / 2) * g.dm;
  const double r2 = l * l + m * m;
  return -r2 / (1.0 + sqrt(1.0 - r2));
}

// Screen phasor exp(+-2 pi i w_k (n - 1)) of pixel (p, q), handed out plane
// by plane (k = 0, 1, ... in order, each once).  The phases w_0 (n - 1) and
// dw (n - 1) are formed and reduced to [-1/2, 1/2] turn in FP64 on both
// paths, and the phasor of plane 0 and the step between planes are taken
// from them with FP64 sincospi; each further plane's phasor is the
// previous one times the step (the planes are equispaced in w).  The FP64
// path advances an FP64 phasor; the FP32 path rounds the seed and step to
// FP32 and advances in FP32 (4 registers of state per pixel): its phase
// error grows by about one FP32 rounding per plane (~2e-6 rad after 32
// planes) and never sees the large unreduced argument.  `odd` adds half a
// turn to the seed: the output centring sign of odd pixels.
template <typename R>
struct Screen {
  cplx<R> ph, step;
  __device__ __forceinline__ void init(const Geo& g, int p, int q, bool conj,
                                       bool odd = false) {
    const double nm1 = n_minus_one(g, p, q);
    const cplx<double> a = turns_phasor(fma(g.w0, nm1, odd ? 0.5 : 0.0));
    const cplx<double> b = turns_phasor(g.dw * nm1);
    ph = {(R)a.re, (R)(conj ? -a.im : a.im)};
    step = {(R)b.re, (R)(conj ? -b.im : b.im)};
  }
  __device__ __forceinline__ cplx<R> next(const Geo&, int) {
    const cplx<R> w = ph;
    ph = cmul(ph, step);
    return w;
  }
};

// The plane sum sum_k F_k ph_0 step^k by Horner's rule, planes taken last
// to first: acc <- acc * step + F_k, and ph_0 * acc once at the end.  The
// same products as handing out ph_k (the contribution of plane k is
// multiplied by the step k times either way), in four fused multiply-adds
// per sample and plane instead of eight.
template <typename R>
__device__ __forceinline__ cplx<R> horner_step(cplx<R> acc, cplx<R> step,
                                               cplx<R> f) {
  return {fma(acc.re, step.re, fma(-acc.im, step.im, f.re)),
          fma(acc.re, step.im, fma(acc.im, step.re, f.im))};
}

// Grid correction of pixel (p, q): 1 / (c psi(f_p) psi(f_q)) from the
// plan's table, or 1 when the plan has none (uniform branch).  Imaging
// multiplies the plane sum by it; degridding multiplies its input image by
// it (the correction is real and diagonal, so it is its own adjoint).
template <typename R>
__device__ __forceinline__ cplx<R> corrected(const Geo& g, int p, int q,
                                             cplx<R> v) {
  if (g.corr == nullptr) return v;
  const R c = (R)(g.corr[p] * g.corr[g.nu + q]);
  return {v.re * c, v.im * c};
}

template <typename R>
__global__ __launch_bounds__(256) void k_wcorrect(const cplx<R>* __restrict__ F,
                                                  cplx<R>* __restrict__ img,
                                                  Geo g) {
  const int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t npix = (int64_t)g.nu * g.nv;
  if (pix >= npix) return;
  const int q = (int)(pix / g.nu), p = (int)(pix - (int64_t)q * g.nu);
  Screen<R> sc;
  sc.init(g, p, q, false);
  cplx<R> acc = {(R)0, (R)0};
  const int64_t src = (int64_t)stack_row(g, q) * g.nu + p;
  for (int k = g.nw - 1; k >= 0; --k)
    acc = horner_step(acc, sc.step, F[(size_t)k * npix + src]);
  img[pix] = cadd(img[pix], corrected(g, p, q, cmul(sc.ph, acc)));
}

// Row transform of every plane + screen + plane sum into image row q.
template <typename R, int LOGN, int NT>
__global__ __launch_bounds__(NT, sizeof(R) == 4 ? 4 : 1) void k_row_screen_sum(
    const cplx<R>* __restrict__ planes, cplx<R>* __restrict__ img, Geo g,
    const cplx<R>* __restrict__ tw, const uint32_t* __restrict__ strips) {
  constexpr int N = 1 << LOGN;
  using L = Stage<R, LOGN, 1, NT, (LOGN / 3) + ((LOGN % 3) ? 1 : 0) - 1>;
  constexpr int IT = L::IT, RAD = L::RAD, NB = L::NB;
  __shared__ cplx<R> lds[lds_line<N>(1)];
  __shared__ cplx<R> s_tab[stage_tw_total(LOGN)];
  const int q = blockIdx.x;
  // Stage twiddles in LDS, the input centring folded into the last stage;
  // the output centring (-1)^p is half a turn in the screen phase (p has
  // the parity of the thread index: NT and NB are even).
  fill_stage_twiddles<R, LOGN>(s_tab, tw, (R)1, true);
  __syncthreads();
  const TableTwiddles<R> twl{s_tab};
  static_assert(NT % 2 == 0 && NB % 2 == 0, "output parity per thread");
  const bool odd = (threadIdx.x & 1) != 0;
  cplx<R> acc[IT][RAD];
  Screen<R> sc[IT][RAD];
#pragma unroll
  for (int it = 0; it < IT; ++it)
#pragma unroll
    for (int r = 0; r < RAD; ++r) {
      const int p = threadIdx.x + it * NT + r * NB;
      acc[it][r] = {(R)0, (R)0};
      if (NB % NT == 0 || threadIdx.x + it * NT < NB)
        sc[it][r].init(g, p, q, false, odd);
    }
  // Row q of the next plane (k - 1) can be loaded into registers while
  // plane k is being transformed, so the HBM reads overlap the LDS stages.
  using F0 = Stage<R, LOGN, 1, NT, 0>;
  constexpr int IT0 = F0::IT, RAD0 = F0::RAD, NB0 = F0::NB;
  // FP32: two workgroups per CU (register-capped) overlap each other's
  // loads, so no register prefetch; FP64 runs one and prefetches.
  constexpr bool kPrefetch = sizeof(R) == 8;
  cplx<R> cur[IT0][RAD0], nxt[IT0][RAD0];
  // Column-strip marks (non-null; used when T is 64, so that the 64
  // samples one wavefront loads lie in one strip): samples of strips that
  // hold no data are not read, since gridding left those columns zero and
  // the column transform kept them so.  The marks of the next plane are
  // loaded (uniform loads, issued together) while plane k is transformed.
  const bool skip = g.T == 64 && NB0 % 64 == 0;
  auto marks = [&](int k, uint32_t (&on)[IT0][RAD0]) {
    const uint32_t* sp = strips + (size_t)(k < g.nw ? k : 0) * g.tiles_u;
#pragma unroll
    for (int it = 0; it < IT0; ++it)
#pragma unroll
      for (int r = 0; r < RAD0; ++r) {
        const uint32_t e = threadIdx.x + it * NT + r * NB0;
        on[it][r] = skip ? sp[uniform_u32(e >> 6)] : 1u;
      }
  };
  auto fetch = [&](int k, const uint32_t (&on)[IT0][RAD0],
                   cplx<R> (&buf)[IT0][RAD0]) {
    const cplx<R>* line = planes + ((size_t)k * g.nv + stack_row(g, q)) * N;
#pragma unroll
    for (int it = 0; it < IT0; ++it)
#pragma unroll
      for (int r = 0; r < RAD0; ++r) {
        const int j = threadIdx.x + it * NT;
        if (NB0 % NT == 0 || j < NB0)
          buf[it][r] = on[it][r] != 0u ? line[j + r * NB0]
                                       : cplx<R>{(R)0, (R)0};
      }
  };
  // Planes last to first (Horner's rule for the screen, horner_step).
  uint32_t on[IT0][RAD0], on_next[IT0][RAD0];
  marks(g.nw - 1, on);
  if (kPrefetch) fetch(g.nw - 1, on, cur);
  for (int k = g.nw - 1; k >= 0; --k) {
    marks(k > 0 ? k - 1 : 0, on_next);
    if (kPrefetch && k > 0) fetch(k - 1, on_next, nxt);
    if (!kPrefetch) fetch(k, on, cur);
    auto ld = [&](int, int, int it, int r) { return cur[it][r]; };
    auto st = [&](int, int, int it, int r, cplx<R> v) {
      acc[it][r] = horner_step(acc[it][r], sc[it][r].step, v);
    };
    fft_line<R, LOGN, 1, NT>(lds, ld, st, twl, (R)1);
    if (kPrefetch) {
#pragma unroll
      for (int it = 0; it < IT0; ++it)
#pragma unroll
        for (int r = 0; r < RAD0; ++r) cur[it][r] = nxt[it][r];
    }
#pragma unroll
    for (int it = 0; it < IT0; ++it)
#pragma unroll
      for (int r = 0; r < RAD0; ++r) on[it][r] = on_next[it][r];
  }
  // Add into the image row: all reads first, then all writes.
  cplx<R>* out = img + (size_t)q * N;
  cplx<R> old[IT][RAD];
#pragma unroll
  for (int it = 0; it < IT; ++it)
#pragma unroll
    for (int r = 0; r < RAD; ++r) {
      const int j = threadIdx.x + it * NT;
      if (NB % NT == 0 || j < NB) old[it][r] = out[j + r * NB];
    }
#pragma unroll
  for (int it = 0; it < IT; ++it)
#pragma unroll
    for (int r = 0; r < RAD; ++r) {
      const int j = threadIdx.x + it * NT;
      if (NB % NT == 0 || j < NB)
        out[j + r * NB] = cadd(
            old[it][r],
            corrected(g, j + r * NB, q, cmul(sc[it][r].ph, acc[it][r])));
    }
}

// Degridding counterpart: image row q times each plane's conjugate screen,
// then the row transform (sign -1), written to row q of every plane.
template <typename R, int LOGN, int NT>
__global__ __launch_bounds__(NT, sizeof(R) == 4 ? 4 : 1) void k_screen_row_bcast(
    const void* __restrict__ img, int img_real, cplx<R>* __restrict__ planes,
    Geo g, const cplx<R>* __restrict__ tw) {
  constexpr int N = 1 << LOGN;
  using F0 = Stage<R, LOGN, 1, NT, 0>;
  constexpr int IT = F0::IT, RAD = F0::RAD, NB = F0::NB;
  __shared__ cplx<R> lds[lds_line<N>(1)];
  __shared__ cplx<R> s_tab[stage_tw_total(LOGN)];
  const int q = blockIdx.x;
  // Stage twiddles in LDS (conjugate: sign -1), the input centring folded
  // into the last stage; the output centring stays on the stores (the
  // column transform that follows centres the other axis).
  fill_stage_twiddles<R, LOGN>(s_tab, tw, (R)-1, true);
  __syncthreads();
  const TableTwiddles<R> twl{s_tab};
  cplx<R> x[IT][RAD];
  Screen<R> sc[IT][RAD];
#pragma unroll
  for (int it = 0; it < IT; ++it)
#pragma unroll
    for (int r = 0; r < RAD; ++r) {
      const int j = threadIdx.x + it * NT;
      x[it][r] = {(R)0, (R)0};
      if (NB % NT == 0 || j < NB) {
        const int p = j + r * NB;
        if (img_real) {
          x[it][r].re = reinterpret_cast<const R*>(img)[(size_t)q * N + p];
        } else {
          x[it][r] = reinterpret_cast<const cplx<R>*>(img)[(size_t)q * N + p];
        }
        x[it][r] = corrected(g, p, q, x[it][r]);
        sc[it][r].init(g, p, q, true);
      }
    }
  for (int k = 0; k < g.nw; ++k) {
    cplx<R>* line = planes + ((size_t)k * g.nv + q) * N;
    auto ld = [&](int, int, int it, int r) {
      const auto w = sc[it][r].next(g, k);
      return cmul(x[it][r], cplx<R>{(R)w.re, (R)w.im});
    };
    auto st = [&](int e, int, int, int, cplx<R> v) { line[e] = checker(v, e); };
    fft_line<R, LOGN, 1, NT>(lds, ld, st, twl, (R)-1);
  }
}

// Degridding, any grid size: plane k = image * conj(screen_k), natural
// row order, one pixel per thread across all planes.
template <typename R>
__global__ __launch_bounds__(256) void k_screen_bcast(
    const void* __restrict__ img, int img_real, cplx<R>* __restrict__ planes,
    Geo g) {
  const int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t npix = (int64_t)g.nu * g.nv;
  if (pix >= npix) return;
  const int q = (int)(pix / g.nu), p = (int)(pix - (int64_t)q * g.nu);
  cplx<R> x = {(R)0, (R)0};
  if (img_real) x.re = reinterpret_cast<const R*>(img)[pix];
  else x = reinterpret_cast<const cplx<R>*>(img)[pix];
  x = corrected(g, p, q, x);
  Screen<R> sc;
  sc.init(g, p, q, true);
  for (int k = 0; k < g.nw; ++k) {
    const auto w = sc.next(g, k);
    planes[(size_t)k * npix + pix] = cmul(x, cplx<R>{(R)w.re, (R)w.im});
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_fill_zero(cplx<R>* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = i; t < n; t += stride) p[t] = cplx<R>{(R)0, (R)0};
}

__global__ __launch_bounds__(256) void k_fill_zero_u32(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = i; t < n; t += stride) p[t] = 0u;
}

// Grid-correction table: thread i < nu gives 1 / (c psi(f_i)) for the u
// axis, thread nu + i gives 1 / psi(f_i) for the v axis.
__global__ __launch_bounds__(256) void k_correction(Geo g, double* corr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.nu + g.nv) return;
  const bool u = i < g.nu;
  const int n = u ? g.nu : g.nv;
  const int idx = u ? i : i - g.nu;
  const double f = (double)(idx - n / 2) / (double)n;
  const double psi = kernel_transform(g.kern, g.K, g.inv2s2, g.es_beta, f);
  corr[i] = 1.0 / ((u ? g.cnorm : 1.0) * psi);
}

template <typename R>
__global__ __launch_bounds__(256) void k_twiddles(cplx<R>* tw, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double sn, cs;
  sincospi(2.0 * (double)i / (double)n, &sn, &cs);
  tw[i] = cplx<R>{(R)cs, (R)sn};
}

// Threads per row transform: enough to cover the N/8 first-stage
// butterflies once, 64..512.
constexpr int row_threads(int logn) {
  return (1 << logn) / 8 < 64 ? 64 : ((1 << logn) / 8 > 512 ? 512 : (1 << logn) / 8);
}

// A whole line of 2^LOGN elements of type R fits one workgroup's LDS.
template <typename R, int LOGN>
constexpr bool line_fits() {
  return lds_line<(1 << LOGN)>(1) * (int)sizeof(cplx<R>) <= 150 * 1024;
}

template <typename R, int LOGN>
bool rows_t(cplx<R>* data, int64_t nrows, const cplx<R>* tw, R s,
            cplx<R>* scratch, const uint32_t* strips, int rows_per_plane,
            int strips_per_row, hipStream_t st) {
  if constexpr (line_fits<R, LOGN>()) {
    constexpr int NT = row_threads(LOGN);
    if (strips == nullptr) {
      hipLaunchKernelGGL((k_fft_rows<R, LOGN, NT, false>),
                         dim3((unsigned)nrows), dim3(NT), 0, st, data, nrows,
                         tw, s, strips, rows_per_plane, strips_per_row);
      return true;
    }
    if constexpr (NT % 64 == 0 && ((1 << LOGN) / 8) % 64 == 0) {
      hipLaunchKernelGGL((k_fft_rows<R, LOGN, NT, true>),
                         dim3((unsigned)nrows), dim3(NT), 0, st, data, nrows,
                         tw, s, strips, rows_per_plane, strips_per_row);
      return true;
    }
    return false;
  } else if constexpr (line_fits<R, LOGN - 1>()) {
    constexpr int NT = row_threads(LOGN - 1);
    if (strips == nullptr) {
      hipLaunchKernelGGL((k_fft_rows_split<R, LOGN - 1, NT, false>),
                         dim3((unsigned)nrows), dim3(NT), 0, st, data, nrows,
                         tw, s, strips, rows_per_plane, strips_per_row);
      return true;
    }
    if constexpr (NT % 64 == 0 && ((1 << (LOGN - 1)) / 8) % 64 == 0) {
      hipLaunchKernelGGL((k_fft_rows_split<R, LOGN - 1, NT, true>),
                         dim3((unsigned)nrows), dim3(NT), 0, st, data, nrows,
                         tw, s, strips, rows_per_plane, strips_per_row);
      return true;
    }
    return false;
  } else if constexpr (line_fits<R, LOGN - 2>()) {
    if (scratch == nullptr || strips != nullptr) return false;
    constexpr int NT = row_threads(LOGN - 2);
    const int64_t g = nrows < kSplitRowGroups ? nrows : kSplitRowGroups;
    hipLaunchKernelGGL((k_fft_rows_splitF<R, LOGN - 2, NT, 4>),
                       dim3((unsigned)(g > 0 ? g : 1)), dim3(NT), 0, st, data,
                       nrows, tw, s, scratch);
    return true;
  } else {
    return false;
  }
}

int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

template <typename R, int LOGN>
bool cols_t(cplx<R>* data, int ncols, int nplanes, const cplx<R>* tw, R s,
            const uint32_t* strips, int strip_w, const uint32_t* tiles,
            const cplx<R>* tstore, const uint32_t* tslot, uint32_t tcap,
            hipStream_t st) {
  if constexpr (LOGN > 12) {
    return false;
  } else {
  constexpr int N = 1 << LOGN;
  constexpr int ELEM = sizeof(cplx<R>);
  // Strips and tile rows are powers of two; a tile table covers at most
  // 64 tile rows (one bit each in a wavefront mask).
  const bool pow2 = strip_w > 0 && (strip_w & (strip_w - 1)) == 0;
  if (!pow2) {
    if (tiles != nullptr) return false;
    strips = nullptr;
  }
  const int log_strip = pow2 ? ilog2(strip_w) : 0;
  if (tiles != nullptr && (N >> log_strip) > 64) return false;
  // Widest column block (<= 16) whose padded N x BC tile fits 150 KiB of
  // LDS (the twiddle tables take the rest).
  constexpr int BCMAX = (150 * 1024) / (lds_line<N>(1) * ELEM);
  constexpr int BC = BCMAX >= 16 ? 16 : (BCMAX >= 8 ? 8 : (BCMAX >= 4 ? 4 : (BCMAX >= 2 ? 2 : 1)));
  constexpr int NT = (N * BC) / 8 < 64 ? 64 : ((N * BC) / 8 > 1024 ? 1024 : (N * BC) / 8);
  const int nb = (ncols / BC) * nplanes;
  const int grid = ((nb + 7) / 8) * 8;
  if constexpr (BC * ELEM < 128 && LOGN >= 10) {
    // Twice the columns per block with the split transform.
    constexpr int BC2 = 2 * BC;
    // FP32: 512 threads (256 registers each: a deeper queue of loads per
    // wavefront beats more wavefronts; measured 25% faster than 1024 at
    // 4096-point columns); FP64: 1024.
    constexpr int CAP = sizeof(R) == 4 ? 512 : 1024;
    constexpr int NT2 = (N / 2 * BC2) / 8 > CAP ? CAP : (N / 2 * BC2) / 8;
    if (ncols % BC2 == 0) {
      const int nb2 = (ncols / BC2) * nplanes;
      if (strip_w % BC2 != 0) {
        if (tiles != nullptr) return false;  // the table cannot be honoured
        strips = nullptr;
      }
      if constexpr (BC2 * ELEM == 64 && NT2 / BC2 == 64 && LOGN >= 7) {
        if (tstore != nullptr) {
          if (tiles == nullptr || strips == nullptr || strip_w != 64)
            return false;
          hipLaunchKernelGGL((k_fft_cols_split<R, LOGN - 1, BC2, NT2, true>),
                             dim3(((nb2 + 7) / 8) * 8), dim3(NT2), 0, st,
                             data, ncols, nplanes, tw, s, strips, log_strip,
                             tiles, tstore, tslot, tcap);
          return true;
        }
      }
      if (tstore != nullptr) return false;
      hipLaunchKernelGGL((k_fft_cols_split<R, LOGN - 1, BC2, NT2, false>),
                         dim3(((nb2 + 7) / 8) * 8), dim3(NT2), 0, st, data,
                         ncols, nplanes, tw, s, strips, log_strip, tiles,
                         (const cplx<R>*)nullptr, (const uint32_t*)nullptr,
                         0u);
      return true;
    }
  }
  if (tstore != nullptr) return false;
  if (strip_w % BC != 0) {
    if (tiles != nullptr) return false;
    strips = nullptr;
  }
  hipLaunchKernelGGL((k_fft_cols<R, LOGN, BC, NT>), dim3(grid), dim3(NT), 0,
                     st, data, ncols, nplanes, tw, s, strips, log_strip, tiles);
  return true;
  }
}

template <typename R, int LOG1, int LOG2, int BC>
bool cols4_bc(cplx<R>* data, int ncols, int nplanes, const cplx<R>* tw, R s,
              const uint32_t* strips, int strip_w, const uint32_t* tiles,
              const cplx<R>* zeros, hipStream_t st) {
  constexpr int NTA = ((1 << LOG1) * BC) / 8;
  constexpr int NTB = ((1 << LOG2) * BC) / 8;
  static_assert(NTA <= 1024 && NTB <= 1024, "step too long for one block");
  const int ncb = ncols / BC;
  const int nba = ncb * (1 << LOG2) * nplanes;
  const int nbb = ncb * (1 << LOG1) * nplanes;
  if (strips != nullptr && strip_w % BC != 0) strips = nullptr;
  if (tiles != nullptr) {
    // Tile counts need strips of 64 columns holding whole blocks.
    if (strips == nullptr || strip_w != 64 || 64 % BC != 0 ||
        zeros == nullptr)
      return false;
    hipLaunchKernelGGL((k_fft_colA<R, LOG1, LOG2, BC, NTA, true>),
                       dim3(((nba + 7) / 8) * 8), dim3(NTA), 0, st, data,
                       ncols, nplanes, tw, s, strips, strip_w, tiles, zeros);
  } else {
    hipLaunchKernelGGL((k_fft_colA<R, LOG1, LOG2, BC, NTA, false>),
                       dim3(((nba + 7) / 8) * 8), dim3(NTA), 0, st, data,
                       ncols, nplanes, tw, s, strips, strip_w, tiles, zeros);
  }
  hipLaunchKernelGGL((k_fft_colB<R, LOG1, LOG2, BC, NTB>),
                     dim3(((nbb + 7) / 8) * 8), dim3(NTB), 0, st, data, ncols,
                     nplanes, tw, s, strips, strip_w);
  return true;
}

template <typename R, int LOGN>
bool cols4_t(cplx<R>* data, int ncols, int nplanes, const cplx<R>* tw, R s,
             const uint32_t* strips, int strip_w, const uint32_t* tiles,
             const cplx<R>* zeros, hipStream_t st) {
  if constexpr (LOGN < 6) {
    return false;
  } else {
    constexpr int LOG1 = LOGN / 2, LOG2 = LOGN - LOG1;
    // 512-byte row segments (64 FP32 or 32 FP64 columns) per workgroup
    // when the grid is that wide (fewer if a step would exceed 1024
    // threads); 16 columns otherwise.
    constexpr int BCW = 512 / (int)sizeof(cplx<R>);
    constexpr int NMAX = (1 << LOG2) > (1 << LOG1) ? (1 << LOG2) : (1 << LOG1);
    constexpr int BC = (NMAX * BCW) / 8 > 1024 ? (8 * 1024) / NMAX : BCW;
    if (ncols >= BC && ncols % BC == 0)
      return cols4_bc<R, LOG1, LOG2, BC>(data, ncols, nplanes, tw, s, strips,
                                         strip_w, tiles, zeros, st);
    return cols4_bc<R, LOG1, LOG2, 16>(data, ncols, nplanes, tw, s, strips,
                                       strip_w, tiles, zeros, st);
  }
}

template <typename R, int LOGN>
bool row_screen_t(const cplx<R>* planes, cplx<R>* img, const Geo& g,
                  const cplx<R>* tw, const uint32_t* strips, hipStream_t st) {
  if constexpr (LOGN > 12) {
    return false;
  } else {
    constexpr int NT = row_threads(LOGN);
    hipLaunchKernelGGL((k_row_screen_sum<R, LOGN, NT>), dim3(g.nv), dim3(NT),
                       0, st, planes, img, g, tw, strips);
    return true;
  }
}

template <typename R, int LOGN>
bool screen_bcast_t(const void* img, int img_real, cplx<R>* planes,
                    const Geo& g, const cplx<R>* tw, hipStream_t st) {
  if constexpr (LOGN > 12) {
    return false;
  } else {
    constexpr int NT = row_threads(LOGN);
    hipLaunchKernelGGL((k_screen_row_bcast<R, LOGN, NT>), dim3(g.nv),
                       dim3(NT), 0, st, img, img_real, planes, g, tw);
    return true;
  }
}

#define WS_LOGN_SWITCH(LOGN_VAR, CALL)                                     \
  switch (LOGN_VAR) {                                                      \
    case 4: { constexpr int LG = 4; CALL; } break;                         \
    case 5: { constexpr int LG = 5; CALL; } break;                         \
    case 6: { constexpr int LG = 6; CALL; } break;                         \
    case 7: { constexpr int LG = 7; CALL; } break;                         \
    case 8: { constexpr int LG = 8; CALL; } break;                         \
    case 9: { constexpr int LG = 9; CALL; } break;                         \
    case 10: { constexpr int LG = 10; CALL; } break;                       \
    case 11: { constexpr int LG = 11; CALL; } break;                       \
    case 12: { constexpr int LG = 12; CALL; } break;                       \
    case 13: { constexpr int LG = 13; CALL; } break;                       \
    case 14: { constexpr int LG = 14; CALL; } break;                       \
    case 15: { constexpr int LG = 15; CALL; } break;                       \
    default: return false;                                                 \
  }

}  // namespace

bool fft_supported(int n, int elem_bytes) {
  // A quarter row must fit one workgroup's LDS (150 KiB with padding).
  return n >= 16 && n <= 32768 && (n & (n - 1)) == 0 &&
         (size_t)(n / 4 + n / 128) * elem_bytes <= 150 * 1024;
}

bool fft_row_needs_scratch(int n, int elem_bytes) {
  // Rows longer than two half-length LDS transforms take the 4-way split.
  return (size_t)(n / 2 + n / 64) * elem_bytes > 150 * 1024;
}

size_t fft_row_scratch_bytes(int n, int elem_bytes) {
  return fft_row_needs_scratch(n, elem_bytes)
             ? (size_t)kSplitRowGroups * n * elem_bytes : 0;
}

// The row kernels for n read by strip marks when one wavefront's 64
// first-stage samples lie in one strip: the one-pass and two-half forms
// at n >= 1024, not the 4-way split.
bool fft_rows_can_mask(int n, int elem_bytes) {
  return n >= 1024 && fft_supported(n, elem_bytes) &&
         !fft_row_needs_scratch(n, elem_bytes);
}

template <typename R>
bool launch_fft_rows(void* data, int n, int64_t nrows, const void* tw, int sign,
                     void* scratch, const uint32_t* strips, int rows_per_plane,
                     hipStream_t st) {
  const int lg = ilog2(n);
  bool ok = false;
  WS_LOGN_SWITCH(lg, (ok = rows_t<R, LG>((cplx<R>*)data, nrows,
                                         (const cplx<R>*)tw, (R)sign,
                                         (cplx<R>*)scratch, strips,
                                         rows_per_plane, n / 64, st)));
  return ok;
}

template <typename R>
bool launch_fft_cols(void* data, int nrows, int ncols, int nplanes,
                     const void* tw, int sign, const uint32_t* strips,
                     int strip_w, const uint32_t* tiles, const void* tstore,
                     const uint32_t* tslot, uint32_t tcap, hipStream_t st) {
  const int lg = ilog2(nrows);
  bool ok = false;
  WS_LOGN_SWITCH(lg, (ok = cols_t<R, LG>((cplx<R>*)data, ncols, nplanes,
                                         (const cplx<R>*)tw, (R)sign, strips,
                                         strip_w, tiles,
                                         (const cplx<R>*)tstore, tslot, tcap,
                                         st)));
  return ok;
}

template <typename R>
bool launch_row_screen_sum(const void* planes, void* img, const Geo& g,
                           const void* tw_u, const uint32_t* strips,
                           hipStream_t st) {
  const int lg = ilog2(g.nu);
  bool ok = false;
  WS_LOGN_SWITCH(lg, (ok = row_screen_t<R, LG>((const cplx<R>*)planes,
                                               (cplx<R>*)img, g,
                                               (const cplx<R>*)tw_u, strips,
                                               st)));
  return ok;
}

template <typename R>
bool launch_screen_row_bcast(const void* img, int img_real, void* planes,
                             const Geo& g, const void* tw_u, hipStream_t st) {
  const int lg = ilog2(g.nu);
  bool ok = false;
  WS_LOGN_SWITCH(lg, (ok = screen_bcast_t<R, LG>(img, img_real,
                                                 (cplx<R>*)planes, g,
                                                 (const cplx<R>*)tw_u, st)));
  return ok;
}

template <typename R>
bool launch_fft_cols4(void* data, int nrows, int ncols, int nplanes,
                      const void* tw, int sign, const uint32_t* strips,
                      int strip_w, const uint32_t* tiles, const void* zeros,
                      hipStream_t st) {
  const int lg = ilog2(nrows);
  bool ok = false;
  WS_LOGN_SWITCH(lg, (ok = cols4_t<R, LG>((cplx<R>*)data, ncols, nplanes,
                                          (const cplx<R>*)tw, (R)sign, strips,
                                          strip_w, tiles,
                                          (const cplx<R>*)zeros, st)));
  return ok;
}

template <typename R>
void launch_unpermute_rows(const void* src, void* dst, const Geo& g,
                           hipStream_t st) {
  const int bx = (g.nu + 255) / 256 < 16 ? (g.nu + 255) / 256 : 16;
  hipLaunchKernelGGL(k_unpermute_rows<R>, dim3(bx, g.nv), dim3(256), 0, st,
                     (const cplx<R>*)src, (cplx<R>*)dst, g);
}

template <typename R>
void launch_screen_bcast(const void* img, int img_real, void* planes,
                         const Geo& g, hipStream_t st) {
  const int64_t npix = (int64_t)g.nu * g.nv;
  hipLaunchKernelGGL(k_screen_bcast<R>, dim3((unsigned)((npix + 255) / 256)),
                     dim3(256), 0, st, img, img_real, (cplx<R>*)planes, g);
}

template <typename R>
void launch_wcorrect(const void* F, void* img, const Geo& g, hipStream_t st) {
  const int64_t npix = (int64_t)g.nu * g.nv;
  hipLaunchKernelGGL(k_wcorrect<R>, dim3((unsigned)((npix + 255) / 256)),
                     dim3(256), 0, st, (const cplx<R>*)F, (cplx<R>*)img, g);
}

template <typename R>
void launch_fill_zero(void* p, int64_t n, hipStream_t st) {
  if (n == 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_zero<R>, dim3((unsigned)blocks), dim3(256), 0, st,
                     (cplx<R>*)p, n);
}

void launch_zero_u32(uint32_t* p, int64_t n, hipStream_t st) {
  if (n == 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_fill_zero_u32, dim3((unsigned)blocks), dim3(256), 0, st,
                     p, n);
}

void launch_correction(const Geo& g, double* corr, hipStream_t st) {
  const int n = g.nu + g.nv;
  hipLaunchKernelGGL(k_correction, dim3((n + 255) / 256), dim3(256), 0, st,
                     g, corr);
}

template <typename R>
void launch_twiddles(void* tw, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_twiddles<R>, dim3((n + 255) / 256), dim3(256), 0, st,
                     (cplx<R>*)tw, n);
}

#define WS_INST(R)                                                            \
  template bool launch_fft_rows<R>(void*, int, int64_t, const void*, int,    \
                                   void*, const uint32_t*, int,            \
                                   hipStream_t);                             \
  template bool launch_fft_cols<R>(void*, int, int, int, const void*, int,   \
                                   const uint32_t*, int, const uint32_t*,    \
                                   const void*, const uint32_t*, uint32_t,   \
                                   hipStream_t);                             \
  template bool launch_row_screen_sum<R>(const void*, void*, const Geo&,     \
                                         const void*, const uint32_t*,       \
                                         hipStream_t);                       \
  template bool launch_screen_row_bcast<R>(const void*, int, void*,          \
                                           const Geo&, const void*,          \
                                           hipStream_t);                     \
  template void launch_wcorrect<R>(const void*, void*, const Geo&,           \
                                   hipStream_t);                             \
  template bool launch_fft_cols4<R>(void*, int, int, int, const void*, int,  \
                                    const uint32_t*, int, const uint32_t*,   \
                                    const void*, hipStream_t);               \
  template void launch_unpermute_rows<R>(const void*, void*, const Geo&,     \
                                         hipStream_t);                       \
  template void launch_screen_bcast<R>(const void*, int, void*, const Geo&,  \
                                       hipStream_t);                         \
  template void launch_fill_zero<R>(void*, int64_t, hipStream_t);           \
  template void launch_twiddles<R>(void*, int, hipStream_t);
WS_INST(float)
WS_INST(double)
#undef WS_INST

}  // namespace ws
