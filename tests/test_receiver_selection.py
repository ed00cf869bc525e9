"""Host check of the GPU receiver selection logic.

The tile kernel usually picks each receiver without dividing: distance
classes are ranked by products with reciprocals under a safety margin, and
near-ties fall back to the eight quotients of Algorithm 1.  Both functions are taken verbatim from the kernel source,
compiled for the host with g++ (IEEE double, no contraction) and compared on
millions of neighbourhoods built to stress ties: random heights, heights
quantised to four values, neighbours one or a few units in the last place
apart, differences near 2^-48 relative, and drops a few units in the last
place apart within and across distance classes (which exercise the exact
fallback), with dx == dy and dx != dy.
"""
from __future__ import annotations

import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNELS = os.path.join(ROOT, "paper_1803_02977_amd", "csrc", "lem_kernels.hip")

PRELUDE = r"""
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#define __device__
#define __forceinline__ inline
#define __noinline__
constexpr uint8_t kSink = 8;
static double fmax_host(double a, double b) { return std::fmax(a, b); }
#define fmax fmax_host
static int __ffs(unsigned x) { return __builtin_ffs((int)x); }
"""

MAIN = r"""
int main(int argc, char** argv) {
  const long n = argc > 1 ? atol(argv[1]) : 1000000;
  std::mt19937_64 rng(7);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  long bad = 0;
  const double dxs[] = {1.0, 30.0, 100.0, 0.1, 3.0};
  for (long t = 0; t < n; ++t) {
    double h[9];
    const int mode = t % 7;
    const double base = U(rng) * 100;
    const double dx = dxs[t % 5], dy = (t % 3 == 0) ? dx : dxs[(t / 5) % 5];
    const double dd = std::sqrt(dx * dx + dy * dy);
    if (mode >= 5) {
      // Drops a few units in the last place apart: mode 5 within each
      // distance class, mode 6 also across classes (diagonal drops scaled
      // by dd/d so that the quotients nearly tie).
      const double hc = 1.0 + U(rng), D = 0.25 + 0.5 * U(rng);
      const double dist[9] = {dd, dy, dd, dx, 0.0, dx, dd, dy, dd};
      for (int k = 0; k < 9; ++k) {
        double drop = (mode == 6) ? D * dist[k] / dx : D;
        const int u = (int)(U(rng) * 5) - 2;
        for (int j = 0; j < (u < 0 ? -u : u); ++j) drop = std::nextafter(drop, u < 0 ? 0.0 : 1e300);
        h[k] = hc - drop;
      }
      h[4] = hc;
    } else
    for (int k = 0; k < 9; ++k) {
      if (mode == 0) h[k] = U(rng);
      else if (mode == 1) h[k] = std::floor(U(rng) * 4);
      else if (mode == 2) h[k] = std::nextafter(base, U(rng) < 0.5 ? -1e300 : 1e300);
      else if (mode == 3) {
        double v = base;
        const int u = (int)(U(rng) * 6);
        for (int j = 0; j < u; ++j) v = std::nextafter(v, 1e300);
        h[k] = v;
      } else h[k] = base + (U(rng) - 0.5) * 1e-12 * base;
    }
    if (mode >= 2 && mode < 5) h[4] = base + std::ldexp((double)(int)(U(rng) * 8), -48) * base;
    RecvConst rk;
    rk.dx = dx; rk.dy = dy; rk.dd = dd;
    rk.inv_dx = 1.0 / dx; rk.inv_dy = 1.0 / dy; rk.inv_dd = 1.0 / dd;
    const uint8_t got = (dx == dy) ? receiver_code_at<true>(h, 4, 3, rk)
                                   : receiver_code_at<false>(h, 4, 3, rk);
    if (got != receiver_code_by_definition(h[4], h[0], h[1], h[2], h[3], h[5], h[6], h[7], h[8],
                                           dx, dy, dd)) ++bad;
  }
  printf("mismatches %ld of %ld\n", bad, n);
  return bad != 0;
}
"""


def test_fast_receiver_selection_equals_definition(tmp_path):
    src = open(KERNELS).read()
    a = src.index("// Step 2 / Algorithm 1 by the definition")
    b = src.index("// F = K*dt*A^m/d and 1 + F")
    prog = tmp_path / "recv.cpp"
    prog.write_text(PRELUDE + src[a:b] + MAIN)
    exe = tmp_path / "recv"
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", str(prog), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe), "3000000"], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "mismatches 0 of 3000000" in out.stdout
