// The V-cycle's relaxation from zero and the residual after it in one launch
// (2D): y = Q(c2 A r + c1 r) and s = Q(A y - r), both in nnqcomp, whose
// output exponents follow from r's metadata alone (Table 1 estimates), so
// one pass over r can quantize y and, from the y values it just computed,
// s. Internal to the library.
#pragma once

#include "kernels.hpp"

namespace bfpk {

struct RelaxResLaunch {
  StarLaunch relax;   // x = r, y operand = r (its centre values), z = y
  StarLaunch res;     // x = y, y operand = r, z = s
  int rows;           // rows of y and s one wave owns
  int64_t* slots;     // 4 int64 per block: the partial reductions of y and s
};

// Whether the two prepared launches fit the fused kernel (2D, saturate
// mode, 32-bit storage, the same grid, the relaxation reading r as its y
// operand, the residual reading the relaxation's output).
bool relax_res_fits(const StarLaunch& relax, const StarLaunch& res);
// Blocks of the launch for `rows` rows per wave.
int64_t relax_res_blocks(int64_t n, int rows);
hipError_t launch_relax_res(const RelaxResLaunch& L, hipStream_t s);

}  // namespace bfpk
