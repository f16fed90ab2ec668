// One translation unit of P7Viterbi kernel instantiations: group width
// HMSV_G and register counts Q in [HMSV_QLO, HMSV_QHI].  The build compiles
// this file once per (G, Q-range) so the instantiations compile in parallel.
#include <utility>
#include "p7_kernel.hpp"

#if !defined(HMSV_G) || !defined(HMSV_QLO) || !defined(HMSV_QHI)
#error "define HMSV_G, HMSV_QLO and HMSV_QHI"
#endif

namespace hmsv {
namespace {

template <int G, int QLO, int... I>
int register_range(std::integer_sequence<int, I...>) {
    static const P7KernelEntry tab[] = {
        P7KernelEntry{G, QLO + I, &launch_p7<G, QLO + I>, &occupancy_p7<G, QLO + I>}...};
    return register_p7_kernels(tab, (int)(sizeof(tab) / sizeof(tab[0])));
}

const int registered = register_range<HMSV_G, HMSV_QLO>(
    std::make_integer_sequence<int, HMSV_QHI - HMSV_QLO + 1>{});

}  // namespace
}  // namespace hmsv
