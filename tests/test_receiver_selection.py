"""Host check of the GPU receiver selection logic.

The tile kernel picks each receiver with three divisions (one per distance
class) plus an exact check of near-ties, instead of the eight quotients of
Algorithm 1.  Both functions are taken verbatim from the kernel source,
compiled for the host with g++ (IEEE double, no contraction) and compared on
millions of neighbourhoods built to stress ties: random heights, heights
quantised to four values, neighbours one or a few units in the last place
apart, and differences near 2^-48 relative, with dx == dy and dx != dy.
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
    const int mode = t % 5;
    const double base = U(rng) * 100;
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
    if (mode >= 2) h[4] = base + std::ldexp((double)(int)(U(rng) * 8), -48) * base;
    const double dx = dxs[t % 5], dy = (t % 3 == 0) ? dx : dxs[(t / 5) % 5];
    const double dd = std::sqrt(dx * dx + dy * dy);
    if (receiver_code(h, 4, 3, dx, dy, dd) != receiver_code_by_definition(h, 4, 3, dx, dy, dd))
      ++bad;
  }
  printf("mismatches %ld of %ld\n", bad, n);
  return bad != 0;
}
"""


def test_three_division_selection_equals_definition(tmp_path):
    src = open(KERNELS).read()
    a = src.index("// Step 2 / Algorithm 1 by the definition")
    b = src.index("// F = K*dt*A^m/d and 1 + F")
    prog = tmp_path / "recv.cpp"
    prog.write_text(PRELUDE + src[a:b] + MAIN)
    exe = tmp_path / "recv"
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", str(prog), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe), "2000000"], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "mismatches 0 of 2000000" in out.stdout
