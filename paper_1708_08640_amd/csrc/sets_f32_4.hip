// Kernel sets of the FP32 reuse contraction for order-4 tensors.
#include "plan.hpp"

namespace s3 {

bool pick_reuse_f32_4(int JP, KernelSet *ks) {
    switch (JP) {
    case 2: *ks = make_set<4, 2, float>(); return true;
    case 4: *ks = make_set<4, 4, float>(); return true;
    case 8: *ks = make_set<4, 8, float>(); return true;
    }
    return false;
}

}  // namespace s3
