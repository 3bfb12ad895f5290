// Host assembly under AddressSanitizer and UndefinedBehaviorSanitizer.
//
// Reads mesh cases from a binary file and runs the library's host assembly on
// each: valid meshes must assemble and satisfy the invariants of the DEC
// operators (K = D0^T H1 D0 symmetric with zero row sums, positive dual areas
// summing to the mesh area, a permutation and its inverse); invalid ones must
// be refused with the expected error code.  Built by the test with g++ and
// -fsanitize=address,undefined, so any out-of-bounds access, use after free,
// overflow or other undefined behaviour in the parsing and assembly of
// arbitrary user meshes aborts the run.
//
// Record layout (little endian): int64 n, int64 t, int32 expect (0: valid,
// negative: that error code, 1: any error), double xy[2n], int32 tri[3t].
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <fstream>
#include <vector>

#include "../../include/dec_bpm.h"
#include "../../paper_2608_03587_amd/csrc/assembly.hpp"

using decbpm::Assembled;
using decbpm::AssemblyInput;

static bool invariants(const Assembled& a, const std::vector<double>& xy, const std::vector<int32_t>& tri,
                       int64_t n, int64_t t, char* why, size_t nwhy) {
  double area = 0, hsum = 0;
  for (int64_t k = 0; k < t; ++k) {
    const int32_t* v = &tri[3 * k];
    const double s = (xy[2 * v[1]] - xy[2 * v[0]]) * (xy[2 * v[2] + 1] - xy[2 * v[0] + 1]) -
                     (xy[2 * v[2]] - xy[2 * v[0]]) * (xy[2 * v[1] + 1] - xy[2 * v[0] + 1]);
    area += 0.5 * std::fabs(s);
  }
  for (int64_t i = 0; i < n; ++i) {
    if (!(a.h0[i] > 0)) return std::snprintf(why, nwhy, "H0[%lld] = %g", (long long)i, a.h0[i]), false;
    hsum += a.h0[i];
  }
  if (std::fabs(hsum - area) > 1e-12 * area) return std::snprintf(why, nwhy, "sum H0 %g vs area %g", hsum, area), false;
  if (int64_t(a.rp.size()) != n + 1) return std::snprintf(why, nwhy, "row pointer size"), false;
  for (int64_t i = 0; i < n; ++i) {
    double rs = 0, diag = 0;
    for (int64_t e = a.rp[i]; e < a.rp[i + 1]; ++e) {
      const int32_t j = a.col[e];
      if (j < 0 || j >= n) return std::snprintf(why, nwhy, "column out of range"), false;
      rs += a.k[e];
      if (j == i) diag = a.k[e];
      // symmetry: find (j, i)
      bool found = false;
      for (int64_t f = a.rp[j]; f < a.rp[j + 1]; ++f)
        if (a.col[f] == i) {
          found = std::fabs(a.k[f] - a.k[e]) <= 1e-12 * (std::fabs(a.k[e]) + 1e-300);
          break;
        }
      if (!found) return std::snprintf(why, nwhy, "K not symmetric at (%lld, %d)", (long long)i, j), false;
    }
    if (std::fabs(rs) > 1e-10 * std::fabs(diag) + 1e-300)
      return std::snprintf(why, nwhy, "K row %lld sums to %g (diag %g)", (long long)i, rs, diag), false;
  }
  if (int64_t(a.perm.size()) != n || int64_t(a.iperm.size()) != n) return std::snprintf(why, nwhy, "perm size"), false;
  for (int64_t i = 0; i < n; ++i)
    if (a.perm[i] < 0 || a.perm[i] >= n || a.iperm[a.perm[i]] != i)
      return std::snprintf(why, nwhy, "perm/iperm not inverse at %lld", (long long)i), false;
  return true;
}

int main(int argc, char** argv) {
  if (argc != 2) {
    std::fprintf(stderr, "usage: host_driver cases.bin\n");
    return 2;
  }
  std::ifstream f(argv[1], std::ios::binary);
  int cases = 0, bad = 0;
  for (;;) {
    int64_t n = 0, t = 0;
    int32_t expect = 0;
    if (!f.read(reinterpret_cast<char*>(&n), 8)) break;
    f.read(reinterpret_cast<char*>(&t), 8);
    f.read(reinterpret_cast<char*>(&expect), 4);
    std::vector<double> xy(size_t(2 * n));
    std::vector<int32_t> tri(size_t(3 * t));
    f.read(reinterpret_cast<char*>(xy.data()), std::streamsize(xy.size() * 8));
    f.read(reinterpret_cast<char*>(tri.data()), std::streamsize(tri.size() * 4));
    std::vector<double> V(size_t(t), 0.25), W(size_t(n), 0.0);
    AssemblyInput in;
    in.xy = xy.data();
    in.n = n;
    in.tri = tri.data();
    in.n_tri = t;
    in.index_tri = V.data();
    in.absorber = W.data();
    int code = 0;
    char why[256] = "";
    try {
      Assembled a = decbpm::assemble(in);
      if (!invariants(a, xy, tri, n, t, why, sizeof why)) code = 99;
      else (void)decbpm::spectral_radius(a, 0.5, 0.0, a.v);
    } catch (const decbpm::Error& e) {
      code = e.code;
      std::snprintf(why, sizeof why, "%s", e.msg.c_str());
    }
    const bool ok = expect == 1 ? code < 0 : code == expect;
    std::printf("case %d n=%lld t=%lld expect=%d got=%d %s %s\n", cases, (long long)n, (long long)t, expect, code,
                ok ? "ok" : "MISMATCH", why);
    bad += !ok;
    ++cases;
  }
  std::printf("%d cases, %d mismatches\n", cases, bad);
  return bad ? 1 : 0;
}
