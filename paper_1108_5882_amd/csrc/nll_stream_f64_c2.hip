// Instantiations of the fused likelihood kernel for double amplitudes, 2 complex per lane.
#include "nll_stream_impl.hpp"

namespace pwa {

hipError_t stream_dispatch_f64_c2(int L, int U, int blocks, const StreamArgs &args,
                                  hipStream_t stream) {
    using namespace stream_detail;
    switch (U) {
        case 1: return dispatch_l<double, 2, 1>(L, blocks, args, stream);
        case 2: return dispatch_l<double, 2, 2>(L, blocks, args, stream);
        default: break;
    }
    return hipErrorInvalidValue;
}

}  // namespace pwa
