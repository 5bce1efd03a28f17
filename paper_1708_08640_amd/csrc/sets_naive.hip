// Kernel sets of the ablation without reuse of partial products (the
// per-entry cost of the paper's Algorithm 2), for the shapes of the tests
// and of the 10M-entry workload only.
#include "plan.hpp"

namespace s3 {

namespace {
template <typename T> bool pick_naive_t(int N, int JP, KernelSet *ks) {
    if (N == 3 && JP == 3) { *ks = make_set<3, 3, T, kNaive>(); return true; }
    if (N == 3 && JP == 4) { *ks = make_set<3, 4, T, kNaive>(); return true; }
    if (N == 3 && JP == 10) { *ks = make_set<3, 10, T, kNaive>(); return true; }
    if (N == 4 && JP == 2) { *ks = make_set<4, 2, T, kNaive>(); return true; }
    return false;
}
}  // namespace

bool pick_naive(bool f64, int N, int JP, KernelSet *ks) {
    return f64 ? pick_naive_t<double>(N, JP, ks) : pick_naive_t<float>(N, JP, ks);
}

}  // namespace s3
