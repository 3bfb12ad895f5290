// Host-side (FP64) mesh ingest and operator assembly for the DEC beam-propagation
// library.  Everything here runs once per mesh in dec_bpm_create.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace decbpm {

// Internal error carrier; converted to a return code at the C ABI.
struct Error {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const std::string& msg);

struct AssemblyInput {
  const double* xy = nullptr;  // [2n]
  int64_t n = 0;
  const int32_t* tri = nullptr;  // [3t]
  int64_t n_tri = 0;
  const double* index_tri = nullptr;  // [t] or null
  const double* absorber = nullptr;   // [n] or null
  const double* chi_tri = nullptr;    // [t] or null
  double p1 = 0.5;
  double beta4 = 0.0;
  double p3 = 0.0, p4 = 0.0;  // coefficients of L^3 and L^4
  int nonlinearity = 0;  // 0 = triangle-averaged (Eq. 14), 1 = lumped
  bool reorder = true;
  // radial perfectly matched layer: sigma(r) = pml_sigma ((r - pml_r0)/(pml_r1 - pml_r0))^2
  // beyond pml_r0 (centre at the origin); pml_sigma == 0: none
  double pml_r0 = 0.0, pml_r1 = 0.0, pml_sigma = 0.0;
};

// Operators in the caller's vertex order (FP64), plus the device vertex order.
struct Assembled {
  int64_t n = 0, n_tri = 0, n_edge = 0;
  std::vector<int32_t> tri;  // counter-clockwise
  std::vector<double> h0;    // diag of H0 (barycentric dual areas)
  std::vector<double> v;     // H0^{-1} H0(V)
  std::vector<double> w;     // absorber
  std::vector<double> chibar;
  // CSR of K = D0^T H1 D0 and of Q^T D Q, diagonal included, columns sorted
  std::vector<int64_t> rp;
  std::vector<int32_t> col;
  std::vector<double> k, qdq;
  // with a PML: the complex-stretched K (same CSR pattern) and dual areas;
  // empty otherwise
  std::vector<double> kp_re, kp_im, h0p_re, h0p_im;
  // device order: perm[i] = caller index of device row i; iperm = inverse
  std::vector<int32_t> perm, iperm;
  double rho = 0.0;  // spectral-radius estimate of H_lin
};

Assembled assemble(const AssemblyInput& in);

// Spectral radius of p1 L + beta4 L^2 + p3 L^3 + p4 L^4 - diag(v) by Lanczos on
// the H0-symmetrised operator (FP64), returned with a small safety factor.
double spectral_radius(const Assembled& a, double p1, double beta4, const std::vector<double>& v, double p3 = 0.0,
                       double p4 = 0.0);

// Hilbert-curve index of (x, y) in [0, 2^order)^2.
uint64_t hilbert_index(uint32_t x, uint32_t y, int order);

}  // namespace decbpm
