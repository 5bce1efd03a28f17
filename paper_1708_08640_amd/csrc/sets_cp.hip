// Kernel sets of the hyper-diagonal (CP) core, FP32 and FP64.
#include "plan.hpp"

namespace s3 {

namespace {
template <typename T> bool pick_cp_t(int N, int JP, KernelSet *ks) {
    if (N == 3) {
        switch (JP) {
        case 3: *ks = make_set<3, 3, T, kCP>(); return true;
        case 4: *ks = make_set<3, 4, T, kCP>(); return true;
        case 8: *ks = make_set<3, 8, T, kCP>(); return true;
        case 10: *ks = make_set<3, 10, T, kCP>(); return true;
        case 12: *ks = make_set<3, 12, T, kCP>(); return true;
        case 16: *ks = make_set<3, 16, T, kCP>(); return true;
        }
    } else if (N == 4) {
        switch (JP) {
        case 2: *ks = make_set<4, 2, T, kCP>(); return true;
        case 4: *ks = make_set<4, 4, T, kCP>(); return true;
        case 8: *ks = make_set<4, 8, T, kCP>(); return true;
        }
    }
    return false;
}
}  // namespace

bool pick_cp(bool f64, int N, int JP, KernelSet *ks) {
    return f64 ? pick_cp_t<double>(N, JP, ks) : pick_cp_t<float>(N, JP, ks);
}

}  // namespace s3
