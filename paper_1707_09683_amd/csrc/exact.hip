// Instantiations of the MSV exact pass (exact_kernel), one per register
// count of its 64-lane groups, qx = 1..kMaxExactQ.
#include <utility>
#include "filter_kernel.hpp"

namespace hmsv {
namespace {

template <int... I>
int register_all(std::integer_sequence<int, I...>) {
    return (register_exact(I + 1, &launch_exact<I + 1>) + ...);
}

const int registered = register_all(std::make_integer_sequence<int, kMaxExactQ>{});

}  // namespace
}  // namespace hmsv
