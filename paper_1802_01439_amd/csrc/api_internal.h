// Helpers shared by the C ABI translation units.
#pragma once

#include <string>

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
int default_conv_nq(int k);
int make_conv_plan(const dg_op_desc* d, ConvPlan& P);

}  // namespace dgmf
