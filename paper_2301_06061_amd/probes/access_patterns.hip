// Memory access-pattern probe for the two transform passes of the imaging
// path (not part of libwstack): what HBM rate a pass can reach for the
// shape of its accesses, independent of its arithmetic.
//
// Stack: 32 planes x 4096 x 4096 8-byte (FP32 complex) elements, row-major
// (buffer A), and a second buffer of the same size (B) in which every block
// of BC columns is stored contiguously (block-major).  A workgroup of 512
// threads moves one block of BC columns x 4096 rows, with one workgroup per
// CU (LDS reserved), 32 loads in flight per thread:
//   SS  strided read, strided write (in place)  - the column pass's shape
//   SC  strided read, contiguous write
//   CS  contiguous read, strided write
//   CC  contiguous read and write (in place)
// for BC = 8 (64-byte row segments, the column pass's block) and BC = 16
// (128-byte segments, one whole L2 line).  Two read-only row patterns:
//   R1  one image row of every plane per workgroup, row-major (the fused
//       row pass's reads), two workgroups per CU
//   R5  the same rows from 8-column blocks (64-byte segments, 256 KB apart)
// Every index stays inside the two buffers.  Prints one JSON object.
#include <hip/hip_runtime.h>
#include <cstdio>

namespace {

constexpr int N = 4096, P = 32;

template <int BC, int MODE>
__global__ __launch_bounds__(512) void k_move(float2* A, float2* B) {
  __shared__ float pad[100 * 256];
  constexpr int NB = N / BC, TPC = 512 / BC, IT = N / TPC;
  constexpr int CH = IT < 32 ? IT : 32;
  const int b = blockIdx.x, plane = b / NB, blk = b % NB;
  const int c = threadIdx.x % BC, jt = threadIdx.x / BC;
  float2* strided = A + (size_t)plane * N * N + (size_t)blk * BC;
  float2* packed = B + ((size_t)plane * NB + blk) * (size_t)N * BC;
  constexpr bool kReadStrided = MODE == 0 || MODE == 1;
  constexpr bool kWriteStrided = MODE == 0 || MODE == 2;
  for (int i0 = 0; i0 < IT; i0 += CH) {
    float2 v[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      const int e = jt + (i0 + i) * TPC;
      v[i] = kReadStrided ? strided[(size_t)e * N + c]
                          : packed[(size_t)e * BC + c];
    }
    pad[threadIdx.x] = v[0].x;
    __syncthreads();
    v[0].x += pad[(threadIdx.x + 1) & 511] * 0.0f;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      const int e = jt + (i0 + i) * TPC;
      v[i].x += 1.0f;
      if (kWriteStrided) strided[(size_t)e * N + c] = v[i];
      else packed[(size_t)e * BC + c] = v[i];
    }
  }
}

template <bool BLOCKED>
__global__ __launch_bounds__(512) void k_rows(const float2* S, float2* out) {
  __shared__ float pad[66 * 256];
  const int q = blockIdx.x;
  float2 acc[8] = {};
  for (int k = 0; k < P; ++k) {
    const float2* pl = S + (size_t)k * N * N;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int p = threadIdx.x + r * 512;
      const float2 v = BLOCKED ? pl[((size_t)(p >> 3) * N + q) * 8 + (p & 7)]
                               : pl[(size_t)q * N + p];
      acc[r].x += v.x;
      acc[r].y += v.y;
    }
    pad[threadIdx.x] = acc[0].x;
    __syncthreads();
    acc[0].x += pad[(threadIdx.x + 1) & 511] * 0.0f;
    __syncthreads();
  }
  float s = 0;
  for (int r = 0; r < 8; ++r) s += acc[r].x + acc[r].y;
  out[(size_t)q * 512 + threadIdx.x] = make_float2(s, 0.0f);
}

template <class F>
float time_ms(F f) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
    return -1.0f;
  f();
  (void)hipEventRecord(a);
  for (int r = 0; r < 5; ++r) f();
  (void)hipEventRecord(b);
  (void)hipEventSynchronize(b);
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms / 5;
}

template <int BC>
void blocks(float2* A, float2* B, double gb, bool& first) {
  const int grid = P * (N / BC);
  const char* names[4] = {"SS", "SC", "CS", "CC"};
  float t[4];
  t[0] = time_ms([&] { hipLaunchKernelGGL((k_move<BC, 0>), dim3(grid), dim3(512), 0, 0, A, B); });
  t[1] = time_ms([&] { hipLaunchKernelGGL((k_move<BC, 1>), dim3(grid), dim3(512), 0, 0, A, B); });
  t[2] = time_ms([&] { hipLaunchKernelGGL((k_move<BC, 2>), dim3(grid), dim3(512), 0, 0, A, B); });
  t[3] = time_ms([&] { hipLaunchKernelGGL((k_move<BC, 3>), dim3(grid), dim3(512), 0, 0, A, B); });
  for (int m = 0; m < 4; ++m) {
    printf("%s\"%s_%dB\": {\"ms\": %.3f, \"tb_s\": %.2f}", first ? "" : ", ",
           names[m], BC * 8, t[m], gb / t[m]);
    first = false;
  }
}

}  // namespace

int main() {
  const size_t n = (size_t)P * N * N;
  float2 *A = nullptr, *B = nullptr, *out = nullptr;
  if (hipMalloc(&A, n * 8) != hipSuccess || hipMalloc(&B, n * 8) != hipSuccess ||
      hipMalloc(&out, (size_t)N * 512 * 8) != hipSuccess) {
    printf("{\"error\": \"hipMalloc failed\"}\n");
    return 1;
  }
  if (hipMemset(A, 0, n * 8) != hipSuccess || hipMemset(B, 0, n * 8) != hipSuccess) {
    printf("{\"error\": \"hipMemset failed\"}\n");
    return 1;
  }
  const double gb = 2.0 * n * 8 / 1e9;  // bytes read + written, GB
  printf("{\"stack\": \"32 x 4096 x 4096 x 8 B\", \"unit\": \"TB/s read+written\", ");
  bool first = true;
  blocks<8>(A, B, gb, first);
  blocks<16>(A, B, gb, first);
  const float r1 = time_ms([&] { hipLaunchKernelGGL(k_rows<false>, dim3(N), dim3(512), 0, 0, A, out); });
  const float r5 = time_ms([&] { hipLaunchKernelGGL(k_rows<true>, dim3(N), dim3(512), 0, 0, B, out); });
  printf(", \"R1_rows_row_major\": {\"ms\": %.3f, \"tb_s\": %.2f}", r1, gb / 2 / r1);
  printf(", \"R5_rows_from_8col_blocks\": {\"ms\": %.3f, \"tb_s\": %.2f}}\n", r5, gb / 2 / r5);
  const hipError_t e = hipDeviceSynchronize();
  (void)hipFree(A);
  (void)hipFree(B);
  (void)hipFree(out);
  return e == hipSuccess ? 0 : 1;
}
