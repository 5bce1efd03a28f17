// Kernel sets with the dense part of the contraction on the matrix cores
// (FP32 or BF16 operands, FP32 parameters), for the shapes it is built for.
#include "plan.hpp"

namespace s3 {

bool pick_mx(bool bf16, int N, int JP, KernelSet *ks) {
    if (N == 4 && JP == 8) {
        *ks = bf16 ? make_set<4, 8, float, kMfma16>() : make_set<4, 8, float, kMfma32>();
        return true;
    }
    if (N == 3 && JP == 16) {
        *ks = bf16 ? make_set<3, 16, float, kMfma16>() : make_set<3, 16, float, kMfma32>();
        return true;
    }
    return false;
}

}  // namespace s3
