// Kernel sets of the FP64 reuse contraction.
#include "plan.hpp"

namespace s3 {

bool pick_reuse_f64(int N, int JP, KernelSet *ks) {
    if (N == 3) {
        switch (JP) {
        case 3: *ks = make_set<3, 3, double>(); return true;
        case 4: *ks = make_set<3, 4, double>(); return true;
        case 8: *ks = make_set<3, 8, double>(); return true;
        case 10: *ks = make_set<3, 10, double>(); return true;
        case 12: *ks = make_set<3, 12, double>(); return true;
        case 16: *ks = make_set<3, 16, double>(); return true;
        }
    } else if (N == 4) {
        switch (JP) {
        case 2: *ks = make_set<4, 2, double>(); return true;
        case 4: *ks = make_set<4, 4, double>(); return true;
        case 8: *ks = make_set<4, 8, double>(); return true;
        }
    }
    return false;
}

}  // namespace s3
