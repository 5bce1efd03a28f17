// Kernel sets of the FP32 reuse contraction for order-3 tensors.
#include "plan.hpp"

namespace s3 {

bool pick_reuse_f32_3(int JP, KernelSet *ks) {
    switch (JP) {
    case 3: *ks = make_set<3, 3, float>(); return true;
    case 4: *ks = make_set<3, 4, float>(); return true;
    case 8: *ks = make_set<3, 8, float>(); return true;
    case 10: *ks = make_set<3, 10, float>(); return true;
    case 12: *ks = make_set<3, 12, float>(); return true;
    case 16: *ks = make_set<3, 16, float>(); return true;
    }
    return false;
}

}  // namespace s3
