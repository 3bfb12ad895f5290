// Host-side (FP64) mesh ingest and DEC operator assembly.
//
// The paper builds L from incidence matrices and a Galerkin Hodge star on
// Whitney 1-forms (Eqs. 8, 9, 11).  Per triangle, D0^T H1 D0 restricted to
// that triangle is the P1 stiffness |t| grad(lambda_a).grad(lambda_b), whose
// closed form is -cot(theta_k)/2 on the edge opposite vertex k; that closed
// form is what is accumulated here, edge by edge.  H0 is the barycentric dual
// area (one third of each incident triangle), H0(V) and H0(chi) are the
// per-triangle pulse stars, and Q^T D Q (Eqs. 13, 14) couples the vertices of
// each triangle with weight chi_t |t| / 9.
#include "assembly.hpp"

#include <algorithm>
#include <cmath>
#include <complex>
#include <numeric>

#include "../../include/dec_bpm.h"

namespace decbpm {

void fail(int code, const std::string& msg) { throw Error{code, msg}; }

uint64_t hilbert_index(uint32_t x, uint32_t y, int order) {
  // Descend the quadrant tree from the coarsest level; at each level the
  // remaining coordinates are reflected/transposed into the orientation of
  // the sub-curve, so consecutive indices stay spatially adjacent.
  const uint32_t side = 1u << order;
  uint64_t d = 0;
  for (uint32_t s = side >> 1; s > 0; s >>= 1) {
    const uint32_t rx = (x & s) ? 1u : 0u;
    const uint32_t ry = (y & s) ? 1u : 0u;
    d += uint64_t(s) * uint64_t(s) * uint64_t((3u * rx) ^ ry);
    if (ry == 0) {
      if (rx == 1) {
        x = side - 1 - x;
        y = side - 1 - y;
      }
      const uint32_t t = x;
      x = y;
      y = t;
    }
  }
  return d;
}

namespace {

struct HalfEdge {
  uint64_t key;  // (min << 32) | max
  int32_t tri;
  int8_t forward;  // 1 if traversed min -> max by the CCW triangle
};

}  // namespace

Assembled assemble(const AssemblyInput& in) {
  if (!in.xy || !in.tri) fail(DEC_BPM_EINVAL, "xy and tri must not be NULL");
  if (in.n < 3 || in.n_tri < 1) fail(DEC_BPM_EINVAL, "need at least 3 vertices and 1 triangle");
  if (in.n >= (int64_t(1) << 31) - 1) fail(DEC_BPM_EINVAL, "too many vertices for 32-bit indices");
  if (!(in.p1 >= 0.0) || !(in.beta4 >= 0.0) || !std::isfinite(in.p1) || !std::isfinite(in.beta4))
    fail(DEC_BPM_EINVAL, "p1 and beta4 must be finite and >= 0");
  if (!std::isfinite(in.p3) || !std::isfinite(in.p4)) fail(DEC_BPM_EINVAL, "p3 and p4 must be finite");
  if (in.nonlinearity != 0 && in.nonlinearity != 1) fail(DEC_BPM_EINVAL, "unknown nonlinearity mode");
  if (!(in.pml_sigma >= 0.0) || !std::isfinite(in.pml_sigma) ||
      (in.pml_sigma > 0.0 && !(in.pml_r0 > 0.0 && in.pml_r1 > in.pml_r0 && std::isfinite(in.pml_r1))))
    fail(DEC_BPM_EINVAL, "PML: need pml_sigma >= 0 and, when it is > 0, 0 < pml_r0 < pml_r1");
  if (in.pml_sigma > 0.0 && in.beta4 != 0.0) fail(DEC_BPM_EINVAL, "PML: not available with the beta4 term");
  const int64_t n = in.n, nt = in.n_tri;
  Assembled a;
  a.n = n;
  a.n_tri = nt;

  double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
  for (int64_t i = 0; i < n; ++i) {
    double x = in.xy[2 * i], y = in.xy[2 * i + 1];
    if (!std::isfinite(x) || !std::isfinite(y)) fail(DEC_BPM_EINVAL, "non-finite vertex coordinate");
    xmin = std::min(xmin, x);
    xmax = std::max(xmax, x);
    ymin = std::min(ymin, y);
    ymax = std::max(ymax, y);
  }
  const double extent = std::max(xmax - xmin, ymax - ymin);
  if (!(extent > 0)) fail(DEC_BPM_EMESH, "all vertices coincide");
  const double area_floor = 1e-14 * extent * extent;

  // orientation, areas, validation
  a.tri.assign(in.tri, in.tri + 3 * nt);
  std::vector<double> area(nt);
  std::vector<char> used(n, 0);
  for (int64_t t = 0; t < nt; ++t) {
    int32_t* v = &a.tri[3 * t];
    for (int k = 0; k < 3; ++k)
      if (v[k] < 0 || v[k] >= n) fail(DEC_BPM_EMESH, "triangle " + std::to_string(t) + " has an index out of range");
    if (v[0] == v[1] || v[1] == v[2] || v[0] == v[2])
      fail(DEC_BPM_EMESH, "triangle " + std::to_string(t) + " repeats a vertex");
    const double* p0 = &in.xy[2 * v[0]];
    const double* p1 = &in.xy[2 * v[1]];
    const double* p2 = &in.xy[2 * v[2]];
    double s = 0.5 * ((p1[0] - p0[0]) * (p2[1] - p0[1]) - (p2[0] - p0[0]) * (p1[1] - p0[1]));
    if (std::fabs(s) <= area_floor) fail(DEC_BPM_EMESH, "triangle " + std::to_string(t) + " has (near) zero area");
    if (s < 0) std::swap(v[1], v[2]);
    area[t] = std::fabs(s);
    used[v[0]] = used[v[1]] = used[v[2]] = 1;
  }
  for (int64_t i = 0; i < n; ++i)
    if (!used[i]) fail(DEC_BPM_EMESH, "vertex " + std::to_string(i) + " is not referenced by any triangle");

  // per-triangle data
  std::vector<double> V(nt, 0.0), chi(nt, 1.0);
  if (in.index_tri)
    for (int64_t t = 0; t < nt; ++t) {
      V[t] = in.index_tri[t];
      if (!std::isfinite(V[t])) fail(DEC_BPM_EINVAL, "non-finite index_tri");
    }
  if (in.chi_tri)
    for (int64_t t = 0; t < nt; ++t) {
      chi[t] = in.chi_tri[t];
      if (!std::isfinite(chi[t])) fail(DEC_BPM_EINVAL, "non-finite chi_tri");
    }
  a.w.assign(n, 0.0);
  if (in.absorber)
    for (int64_t i = 0; i < n; ++i) {
      a.w[i] = in.absorber[i];
      if (!std::isfinite(a.w[i]) || a.w[i] < 0) fail(DEC_BPM_EINVAL, "absorber must be finite and >= 0");
    }

  // edges: sort the 3T directed half-edges by their undirected key
  std::vector<HalfEdge> he(3 * nt);
  for (int64_t t = 0; t < nt; ++t) {
    const int32_t* v = &a.tri[3 * t];
    for (int k = 0; k < 3; ++k) {
      uint32_t u = v[k], w = v[(k + 1) % 3];
      uint32_t lo = std::min(u, w), hi = std::max(u, w);
      he[3 * t + k] = HalfEdge{(uint64_t(lo) << 32) | hi, int32_t(t), int8_t(u < w)};
    }
  }
  std::sort(he.begin(), he.end(), [](const HalfEdge& x, const HalfEdge& y) {
    return x.key < y.key || (x.key == y.key && x.tri < y.tri);
  });
  struct Edge {
    int32_t i, j;
    double k, q;
  };
  std::vector<Edge> edges;
  edges.reserve(3 * nt / 2 + 16);
  for (size_t s = 0; s < he.size();) {
    size_t e = s + 1;
    while (e < he.size() && he[e].key == he[s].key) ++e;
    if (e - s > 2) fail(DEC_BPM_EMESH, "an edge is shared by more than two triangles (non-manifold)");
    if (e - s == 2 && he[s].forward == he[s + 1].forward)
      fail(DEC_BPM_EMESH, "two triangles traverse a shared edge in the same direction (overlap or fold)");
    Edge ed{int32_t(he[s].key >> 32), int32_t(he[s].key & 0xffffffffu), 0.0, 0.0};
    for (size_t r = s; r < e; ++r) {
      int32_t t = he[r].tri;
      const int32_t* v = &a.tri[3 * t];
      int32_t o = v[0] + v[1] + v[2] - ed.i - ed.j;  // vertex opposite the edge
      const double* pi = &in.xy[2 * ed.i];
      const double* pj = &in.xy[2 * ed.j];
      const double* po = &in.xy[2 * o];
      double dot = (pi[0] - po[0]) * (pj[0] - po[0]) + (pi[1] - po[1]) * (pj[1] - po[1]);
      double cot = dot / (2.0 * area[t]);
      ed.k += -0.5 * cot;
      ed.q += chi[t] * area[t] / 9.0;
    }
    edges.push_back(ed);
    s = e;
  }
  a.n_edge = int64_t(edges.size());

  // vertex quantities
  a.h0.assign(n, 0.0);
  std::vector<double> h0V(n, 0.0), h0chi(n, 0.0), qdiag(n, 0.0);
  for (int64_t t = 0; t < nt; ++t)
    for (int k = 0; k < 3; ++k) {
      int32_t p = a.tri[3 * t + k];
      a.h0[p] += area[t] / 3.0;
      h0V[p] += V[t] * area[t] / 3.0;
      h0chi[p] += chi[t] * area[t] / 3.0;
      qdiag[p] += chi[t] * area[t] / 9.0;
    }
  a.v.resize(n);
  a.chibar.resize(n);
  for (int64_t p = 0; p < n; ++p) {
    a.v[p] = h0V[p] / a.h0[p];
    a.chibar[p] = h0chi[p] / a.h0[p];
  }

  // CSR with the diagonal; K_pp = -sum of the row's off-diagonals
  std::vector<int64_t> deg(n, 1);
  for (const Edge& e : edges) {
    deg[e.i]++;
    deg[e.j]++;
  }
  a.rp.assign(n + 1, 0);
  for (int64_t p = 0; p < n; ++p) a.rp[p + 1] = a.rp[p] + deg[p];
  const int64_t nnz = a.rp[n];
  a.col.assign(nnz, 0);
  a.k.assign(nnz, 0.0);
  a.qdq.assign(nnz, 0.0);
  std::vector<int64_t> fillp(a.rp.begin(), a.rp.end() - 1);
  for (int64_t p = 0; p < n; ++p) {
    a.col[fillp[p]] = int32_t(p);
    a.qdq[fillp[p]] = in.nonlinearity == 0 ? qdiag[p] : h0chi[p];
    fillp[p]++;
  }
  std::vector<double> ksum(n, 0.0);
  for (const Edge& e : edges) {
    int64_t s1 = fillp[e.i]++, s2 = fillp[e.j]++;
    a.col[s1] = e.j;
    a.col[s2] = e.i;
    a.k[s1] = a.k[s2] = e.k;
    a.qdq[s1] = a.qdq[s2] = in.nonlinearity == 0 ? e.q : 0.0;
    ksum[e.i] += e.k;
    ksum[e.j] += e.k;
  }
  for (int64_t p = 0; p < n; ++p) {
    a.k[a.rp[p]] = -ksum[p];
    // sort the row by column
    int64_t b = a.rp[p], en = a.rp[p + 1];
    std::vector<int64_t> idx(en - b);
    std::iota(idx.begin(), idx.end(), b);
    std::sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) { return a.col[x] < a.col[y]; });
    std::vector<int32_t> c2(idx.size());
    std::vector<double> k2(idx.size()), q2(idx.size());
    for (size_t r = 0; r < idx.size(); ++r) {
      c2[r] = a.col[idx[r]];
      k2[r] = a.k[idx[r]];
      q2[r] = a.qdq[idx[r]];
    }
    std::copy(c2.begin(), c2.end(), a.col.begin() + b);
    std::copy(k2.begin(), k2.end(), a.k.begin() + b);
    std::copy(q2.begin(), q2.end(), a.qdq.begin() + b);
  }

  // Perfectly matched layer: radial complex stretching r~ = r + i S(r),
  // S' = sigma.  With s_r = 1 + i sigma and s_t = r~ / r, the stretched
  // Laplacian is div(Lambda grad) / (s_r s_t), Lambda = (s_t/s_r) r r^T +
  // (s_r/s_t) t t^T.  Per triangle (stretch taken at the centroid) the P1
  // stiffness |t| grad(lambda_a)^T Lambda grad(lambda_b) is D0^T H1 D0 with the
  // stretched Galerkin H1, and the dual areas pick up s_r s_t.
  if (in.pml_sigma > 0.0) {
    using cd = std::complex<double>;
    const double r0 = in.pml_r0, r1 = in.pml_r1, sm = in.pml_sigma;
    std::vector<cd> kp(nnz, cd(0.0)), h0p(n, cd(0.0));
    auto slot = [&](int32_t p, int32_t q) {
      const int32_t* b = a.col.data() + a.rp[p];
      const int32_t* e = a.col.data() + a.rp[p + 1];
      return a.rp[p] + (std::lower_bound(b, e, q) - b);
    };
    for (int64_t t = 0; t < nt; ++t) {
      const int32_t* v = &a.tri[3 * t];
      double P[3][2];
      for (int k = 0; k < 3; ++k) {
        P[k][0] = in.xy[2 * v[k]];
        P[k][1] = in.xy[2 * v[k] + 1];
      }
      const double cx = (P[0][0] + P[1][0] + P[2][0]) / 3.0, cy = (P[0][1] + P[1][1] + P[2][1]) / 3.0;
      const double rc = std::hypot(cx, cy);
      cd s_r(1.0, 0.0), s_t(1.0, 0.0);
      if (rc > r0) {
        const double u = (rc - r0) / (r1 - r0);
        s_r = cd(1.0, sm * u * u);
        s_t = cd(1.0, sm * (r1 - r0) * u * u * u / 3.0 / rc);
      }
      const double ex = rc > 0 ? cx / rc : 1.0, ey = rc > 0 ? cy / rc : 0.0;
      const cd ar = s_t / s_r, at = s_r / s_t;  // radial and azimuthal weights
      const cd L00 = ar * ex * ex + at * ey * ey, L11 = ar * ey * ey + at * ex * ex, L01 = (ar - at) * ex * ey;
      const double A2 = (P[1][0] - P[0][0]) * (P[2][1] - P[0][1]) - (P[2][0] - P[0][0]) * (P[1][1] - P[0][1]);
      double g[3][2];
      for (int k = 0; k < 3; ++k) {
        const double* pb = P[(k + 1) % 3];
        const double* pc = P[(k + 2) % 3];
        g[k][0] = (pb[1] - pc[1]) / A2;
        g[k][1] = (pc[0] - pb[0]) / A2;
      }
      for (int k = 0; k < 3; ++k) h0p[v[k]] += area[t] / 3.0 * s_r * s_t;
      for (int k = 0; k < 3; ++k)
        for (int l = k + 1; l < 3; ++l) {
          const cd kk = area[t] * (g[k][0] * (L00 * g[l][0] + L01 * g[l][1]) + g[k][1] * (L01 * g[l][0] + L11 * g[l][1]));
          kp[slot(v[k], v[l])] += kk;
          kp[slot(v[l], v[k])] += kk;
          kp[slot(v[k], v[k])] -= kk;  // rows sum to zero (K 1 = 0)
          kp[slot(v[l], v[l])] -= kk;
        }
    }
    a.kp_re.resize(nnz);
    a.kp_im.resize(nnz);
    for (int64_t e = 0; e < nnz; ++e) {
      a.kp_re[e] = kp[e].real();
      a.kp_im[e] = kp[e].imag();
    }
    a.h0p_re.resize(n);
    a.h0p_im.resize(n);
    for (int64_t p = 0; p < n; ++p) {
      a.h0p_re[p] = h0p[p].real();
      a.h0p_im[p] = h0p[p].imag();
    }
  }

  // device vertex order: Hilbert curve over the bounding square
  a.perm.resize(n);
  std::iota(a.perm.begin(), a.perm.end(), 0);
  if (in.reorder) {
    const int order = 16;
    const double scale = (double((1u << order) - 1)) / extent;
    std::vector<uint64_t> key(n);
    for (int64_t i = 0; i < n; ++i) {
      uint32_t qx = uint32_t(std::lround((in.xy[2 * i] - xmin) * scale));
      uint32_t qy = uint32_t(std::lround((in.xy[2 * i + 1] - ymin) * scale));
      key[i] = hilbert_index(qx, qy, order);
    }
    std::stable_sort(a.perm.begin(), a.perm.end(), [&](int32_t x, int32_t y) { return key[x] < key[y]; });
  }
  a.iperm.resize(n);
  for (int64_t i = 0; i < n; ++i) a.iperm[a.perm[i]] = int32_t(i);

  a.rho = spectral_radius(a, in.p1, in.beta4, a.v, in.p3, in.p4);
  return a;
}

namespace {

// Number of eigenvalues of the symmetric tridiagonal (alpha, beta) below x (Sturm count).
int sturm_count(const std::vector<double>& al, const std::vector<double>& be, double x) {
  int c = 0;
  double d = 1.0;
  for (size_t i = 0; i < al.size(); ++i) {
    double b2 = i ? be[i - 1] * be[i - 1] : 0.0;
    d = al[i] - x - (i ? b2 / d : 0.0);
    if (d == 0.0) d = 1e-300;
    if (d < 0) ++c;
  }
  return c;
}

}  // namespace

double spectral_radius(const Assembled& a, double p1, double beta4, const std::vector<double>& v, double p3,
                       double p4) {
  const int64_t n = a.n;
  std::vector<double> s(n), is(n);
  for (int64_t p = 0; p < n; ++p) {
    s[p] = std::sqrt(a.h0[p]);
    is[p] = 1.0 / s[p];
  }
  // B = H0^{-1/2} K H0^{-1/2};  S = p1 B + beta4 B^2 + p3 B^3 + p4 B^4 - diag(v)   (symmetric)
  auto applyB = [&](const std::vector<double>& x, std::vector<double>& y) {
    for (int64_t p = 0; p < n; ++p) {
      double acc = 0.0;
      for (int64_t r = a.rp[p]; r < a.rp[p + 1]; ++r) acc += a.k[r] * is[a.col[r]] * x[a.col[r]];
      y[p] = is[p] * acc;
    }
  };
  std::vector<double> t1(n), t2(n);
  const double c[4] = {p1, beta4, p3, p4};
  const int deg = p4 != 0.0 ? 4 : (p3 != 0.0 ? 3 : (beta4 != 0.0 ? 2 : 1));
  auto applyS = [&](const std::vector<double>& x, std::vector<double>& y) {
    for (int64_t p = 0; p < n; ++p) y[p] = -v[p] * x[p];
    applyB(x, t1);
    for (int k = 0; k < deg; ++k) {
      if (k) {
        applyB(t1, t2);
        t1.swap(t2);
      }
      if (c[k] != 0.0)
        for (int64_t p = 0; p < n; ++p) y[p] += c[k] * t1[p];
    }
  };
  const int kmax = int(std::min<int64_t>(n, 120));
  std::vector<double> q(n), qprev(n, 0.0), z(n), al, be;
  // deterministic start vector with content in every mode
  uint64_t st = 0x9E3779B97F4A7C15ull;
  double nrm = 0.0;
  for (int64_t p = 0; p < n; ++p) {
    st ^= st << 13;
    st ^= st >> 7;
    st ^= st << 17;
    q[p] = double(st >> 11) / double(1ull << 53) - 0.5;
    nrm += q[p] * q[p];
  }
  nrm = std::sqrt(nrm);
  for (auto& x : q) x /= nrm;
  const bool full_reorth = n <= 4096;
  std::vector<std::vector<double>> basis;
  double bprev = 0.0;
  for (int k = 0; k < kmax; ++k) {
    if (full_reorth) basis.push_back(q);
    applyS(q, z);
    double alpha = 0.0;
    for (int64_t p = 0; p < n; ++p) alpha += q[p] * z[p];
    for (int64_t p = 0; p < n; ++p) z[p] -= alpha * q[p] + bprev * qprev[p];
    if (full_reorth)
      for (const auto& b : basis) {
        double c = 0.0;
        for (int64_t p = 0; p < n; ++p) c += b[p] * z[p];
        for (int64_t p = 0; p < n; ++p) z[p] -= c * b[p];
      }
    double beta = 0.0;
    for (int64_t p = 0; p < n; ++p) beta += z[p] * z[p];
    beta = std::sqrt(beta);
    al.push_back(alpha);
    if (beta < 1e-13 * std::fabs(alpha) || k == kmax - 1) break;
    be.push_back(beta);
    qprev = q;
    for (int64_t p = 0; p < n; ++p) q[p] = z[p] / beta;
    bprev = beta;
  }
  be.resize(al.size() > 0 ? al.size() - 1 : 0);
  // extreme eigenvalues of the tridiagonal by bisection on the Sturm count
  double lo = INFINITY, hi = -INFINITY;
  for (size_t i = 0; i < al.size(); ++i) {
    double r = (i ? std::fabs(be[i - 1]) : 0.0) + (i + 1 < al.size() ? std::fabs(be[i]) : 0.0);
    lo = std::min(lo, al[i] - r);
    hi = std::max(hi, al[i] + r);
  }
  const int m = int(al.size());
  auto kth = [&](int kidx) {  // kidx-th smallest eigenvalue (0-based)
    double l = lo, h = hi;
    for (int it = 0; it < 200; ++it) {
      double mid = 0.5 * (l + h);
      if (sturm_count(al, be, mid) > kidx)
        h = mid;
      else
        l = mid;
    }
    return 0.5 * (l + h);
  };
  double emin = kth(0), emax = kth(m - 1);
  double rho = std::max(std::fabs(emin), std::fabs(emax));
  return full_reorth ? rho * 1.0001 : rho * 1.01;
}

}  // namespace decbpm
