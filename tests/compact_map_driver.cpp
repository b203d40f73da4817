// Host check of the compact Krylov-vector layout (CMap in sp_internal.h): on
// several grids, the map from compact entries to canonical ones is strictly
// increasing (so one-to-one), lands exactly on the entries of the packed real
// vector space (no x or z Nyquist entry, the m_z = 0 plane at m_x <= nx/2 - 1
// only), covers all of them, and gives each m_z = 0 entry with 0 < m_x < nx/2
// the canonical index of its conjugate partner at -m_x. Exit status 0 when
// every check holds.
#include <cstdio>

#include "sp_internal.h"

static int fail(const char* what, int nx, int ny, int nz) {
  std::fprintf(stderr, "check failed: %s (nx %d ny %d nz %d)\n", what, nx, ny, nz);
  return 1;
}

int main() {
  const int grids[][3] = {{4, 5, 4},   {8, 9, 8},    {12, 20, 12}, {16, 17, 16},
                          {8, 64, 8},  {48, 65, 48}, {6, 7, 10},   {96, 97, 96}};
  for (const auto& g : grids) {
    const int nx = g[0], ny = g[1], nz = g[2];
    sp::Dims d{};
    d.nx = nx;
    d.ny = ny;
    d.nz = nz;
    d.nzh = nz / 2 + 1;
    const sp::CMap m = sp::compact_map(d);
    const int nzh = d.nzh;
    long expect = 0;
    for (int c = 0; c < 3; ++c)
      for (int mx = 0; mx < nx; ++mx)
        for (int kz = 0; kz < nzh; ++kz) {
          const bool kept = mx != nx / 2 && kz != nzh - 1 && !(kz == 0 && mx > nx / 2);
          if (kept) expect += ny;
        }
    if (m.len != expect) return fail("length", nx, ny, nz);
    int prev = -1;
    for (int k = 0; k < m.len; ++k) {
      int mir = -2;
      const int ci = m.canon(k, &mir);
      if (ci <= prev) return fail("strictly increasing", nx, ny, nz);
      prev = ci;
      const int n = ci % ny;
      const int kz = (ci / ny) % nzh;
      const int mx = (ci / (ny * nzh)) % nx;
      const int c = ci / (ny * nzh * nx);
      if (c < 0 || c > 2) return fail("component", nx, ny, nz);
      if (mx == nx / 2 || kz == nzh - 1 || (kz == 0 && mx > nx / 2))
        return fail("entry outside the packed space", nx, ny, nz);
      const int want = (kz == 0 && mx > 0) ? ((c * nx + (nx - mx)) * nzh) * ny + n : -1;
      if (mir != want) return fail("mirror", nx, ny, nz);
    }
  }
  std::puts("compact map: all checks passed");
  return 0;
}
