// Host-side audit of the reduction grids (no GPU needed): for each problem
// size read from stdin ("dim p n1 n2 n3" per line), every kernel shape a
// context can run -- FD tile counts 1..8, fused passes on and off, tiled
// products on, off and by size, the four precisions, A products with 1, 2, 4
// rows per thread and the tile shapes picked for 64, 80 and 160 KB of LDS --
// must write at most partial_capacity() block partials per sum, the size the
// library gives its partial-sum buffer.  Uses the library's own grid
// functions (linked from libigafd.so).  Prints one line per violation and
// "OK <count>" at the end; exit status 1 on any violation.
#include <cstdio>
#include <string>

#include "internal.h"

int main() {
  int dim, p, n1, n2, n3, checked = 0, bad = 0;
  while (std::scanf("%d %d %d %d %d", &dim, &p, &n1, &n2, &n3) == 5) {
    igafd_ctx c;
    c.dim = dim;
    c.p = p;
    c.n[0] = n1;
    c.n[1] = n2;
    c.n[2] = dim == 3 ? n3 : 1;
    c.N = (long long)c.n[0] * c.n[1] * c.n[2];
    c.npartial = igafd::partial_capacity(&c);
    const long long vb = (c.N + igafd::kBlock - 1) / igafd::kBlock;
    auto fail = [&](const char* what, long long got) {
      std::printf("VIOLATION %s: dim %d p %d n %d %d %d: %lld partials > capacity %d\n", what, dim, p, n1, n2, n3,
                  got, c.npartial);
      ++bad;
    };
    if (vb > c.npartial) fail("vector kernels", vb);
    if ((2 * (long long)c.npartial - 3) / 3 < 1) fail("spectral bounds", 0);
    for (int tiles = 1; tiles <= 8; ++tiles)
      for (int fused = 0; fused <= 1; ++fused)
        for (int gemm = -1; gemm <= 1; ++gemm)
          for (int prec = IGAFD_FP64; prec <= IGAFD_BF16X3; ++prec) {
            c.fd_tiles = tiles;
            c.fd_fused = fused;
            c.fd_gemm = gemm;
            const int fb = igafd::fd_dot_blocks(&c, prec);
            ++checked;
            if (fb > c.npartial) fail("FD apply", fb);
          }
    c.fd_gemm = -1;
    // A products: row-parallel kernel with R rows per thread, tiled shapes
    for (int R : {1, 2, 4}) {
      c.spmv_rows = R;
      c.tile_b2 = c.tile_b3 = 0;
      const int sb = igafd::spmv_blocks(&c);
      ++checked;
      if (sb > c.npartial) fail("A product (rows)", sb);
    }
    for (long long lim : {64LL * 1024, igafd::kTileLdsDefault, 160LL * 1024}) {
      int b2 = 0, b3 = 0;
      if (!igafd::spmv_pick_tile(&c, lim, &b2, &b3)) continue;
      c.tile_b2 = b2;
      c.tile_b3 = b3;
      const int sb = igafd::spmv_blocks(&c);
      ++checked;
      if (sb > c.npartial) fail("A product (tiles)", sb);
    }
  }
  std::printf("%s %d\n", bad ? "FAILED" : "OK", checked);
  return bad ? 1 : 0;
}
