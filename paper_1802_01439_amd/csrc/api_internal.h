// Helpers shared by the C ABI translation units.
#pragma once

#include <cstring>
#include <string>
#include <vector>

#include "basis1d.h"
#include "dgmf.h"
#include "ops.h"

namespace dgmf {

constexpr int kMaxDegree = 11;
constexpr int kMaxNq = 32;

int fail(int code, const std::string& msg);
int ok();
int hip_fail(hipError_t e, const char* where);
const Basis1D& basis(int k, int m);
int validate_desc(const dg_op_desc* d);
long long num_elements(const dg_op_desc* d);
long long dofs_per_element(const dg_op_desc* d);
bool overlaps(const void* a, size_t na, const void* b, size_t nb);
MeshArgs mesh_args(const dg_op_desc* d);
LaplacePlan make_laplace_plan(const dg_op_desc* d, int n_comp);
double cell_volume(const dg_op_desc* d);
// M1^-1 of the 1D LGL mass on [0,1] (row major, n x n)
std::vector<double> inverse_mass_1d(int k);
ProjPlan make_proj_plan(const dg_op_desc* d);
DivPlan make_div_plan(const dg_op_desc* d);
// lambda_max bound of D^-1 A for the SIPG form of d (n_comp = 1): 1.1 x the
// largest Ritz value of 25 Lanczos steps, kept per operator (cg.cpp)
int laplace_lambda_max(const dg_op_desc* d, bool project, void* hip_stream, double* lmax);

// FP64 CG with one V-cycle (T = cycle precision, DG_F64 or DG_F32) per
// iteration, stopping at |r| <= max(rtol |b - mean b|, atol); the body of
// dg_gmg_cg_solve (which passes atol = 0 and true_residual).  Without
// true_residual the report's true_rel_res is NaN and the operator apply and
// residual that form it are skipped (callers that read iteration counts).
int gmg_cg_solve(const dg_op_desc* desc, int levels, int degree, double smoothing_range, int coarse_degree,
                 const double* lambda_max, int cycle_dtype, const double* b, double* x, double rtol, double atol,
                 int max_iter, dg_cg_report* report, void* hip_stream, bool true_residual = true);
// dg_mass_pcg_solve with the same true_residual switch
int mass_pcg_solve(const dg_op_desc* desc, int32_t op, double mass_factor, const double* tau_d, const double* tau_c,
                   const double* b, double* x, double rtol, int32_t max_iter, dg_cg_report* report,
                   void* hip_stream, bool true_residual);
int default_conv_nq(int k);
int make_conv_plan(const dg_op_desc* d, ConvPlan& P);

}  // namespace dgmf

namespace dgmf {

// Device copy of a small constant table (1D matrices of one operator
// configuration), uploaded once per (key, device) and kept until exit.
// Kernels read it with uniform addresses through the scalar cache.
const void* device_table(const std::string& key, const void* host, size_t bytes, hipError_t* err);

// Content-addressed variant: the key is the table's size and a 64-bit hash
// of its bytes (FNV-1a steps over 8-byte words, each followed by a
// shift-xor so that high bits reach the low ones; a byte-wise pass took
// microseconds per call for the tables of the high degrees).
template <typename Tab>
const Tab* device_table_of(const char* kind, const Tab& host, hipError_t* err) {
  unsigned long long h = 1469598103934665603ULL;
  const unsigned char* p = reinterpret_cast<const unsigned char*>(&host);
  size_t i = 0;
  for (; i + 8 <= sizeof(Tab); i += 8) {
    unsigned long long w;
    std::memcpy(&w, p + i, 8);
    h = (h ^ w) * 1099511628211ULL;
    h ^= h >> 29;
  }
  for (; i < sizeof(Tab); ++i) h = (h ^ p[i]) * 1099511628211ULL;
  const std::string key = std::string(kind) + ":" + std::to_string(sizeof(Tab)) + ":" + std::to_string(h);
  return static_cast<const Tab*>(device_table(key, &host, sizeof(Tab), err));
}

}  // namespace dgmf
