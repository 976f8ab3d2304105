// Host build of the library's placement and binning logic (ws_common.h),
// for CPU tests: reads a geometry line and float64 (u, v, w) triples, and
// writes, per visibility, "ok i0 j0 k key dropped", then, per tile, its
// gridding key segments "t n lo0 hi0 lo1 hi1 ...".
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "ws_common.h"

int main(int argc, char** argv) {
  if (argc != 3) {
    std::fprintf(stderr, "usage: %s geometry.txt uvw.f64\n", argv[0]);
    return 2;
  }
  ws::Geo g{};
  FILE* fg = std::fopen(argv[1], "r");
  if (!fg) return 3;
  if (std::fscanf(fg, "%d %d %d %d %d %lf %lf %lf %lf", &g.nu, &g.nv, &g.nw,
                  &g.K, &g.T, &g.fov_l, &g.fov_m, &g.w_min, &g.dw) != 9)
    return 4;
  std::fclose(fg);
  g.h = (g.K - 1) / 2;
  g.tiles_u = g.nu / g.T;
  g.tiles_v = g.nv / g.T;
  g.ntiles = g.tiles_u * g.tiles_v * g.nw;
  FILE* fu = std::fopen(argv[2], "rb");
  if (!fu) return 5;
  std::vector<double> uvw;
  double buf[3];
  while (std::fread(buf, sizeof(double), 3, fu) == 3)
    uvw.insert(uvw.end(), buf, buf + 3);
  std::fclose(fu);
  const size_t m = uvw.size() / 3;
  for (size_t i = 0; i < m; ++i) {
    double x, y;
    int i0 = 0, j0 = 0, k = 0;
    const bool ok = ws::place(g, uvw[3 * i], uvw[3 * i + 1], uvw[3 * i + 2],
                              x, y, i0, j0, k);
    const unsigned key = ok ? ws::bin_key(g, i0, j0, k) : ws::kNoKey;
    const int dropped = ok ? g.K * g.K - ws::taps_on_grid(g, i0, j0) : g.K * g.K;
    const unsigned cell = ok ? ws::pack_cell(i0, j0) : 0u;
    const int ri = ok ? ws::cell_i(cell) : 0, rj = ok ? ws::cell_j(cell) : 0;
    std::printf("%d %d %d %d %u %d %d %d\n", ok ? 1 : 0, i0, j0, k, key,
                dropped, ri, rj);
  }
  for (int t = 0; t < g.ntiles; ++t) {
    unsigned lo[ws::kSegments], hi[ws::kSegments];
    ws::tile_segments(g, t, lo, hi);
    const int n = ws::kSegments;
    std::printf("T %d %d", t, n);
    for (int s = 0; s < n; ++s) std::printf(" %u %u", lo[s], hi[s]);
    std::printf("\n");
  }
  return 0;
}
