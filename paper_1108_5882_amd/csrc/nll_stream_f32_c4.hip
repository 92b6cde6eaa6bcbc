// Instantiations of the fused likelihood kernel for float amplitudes, 4 complex per lane.
#include "nll_stream_impl.hpp"

namespace pwa {

hipError_t stream_dispatch_f32_c4(int L, int U, int blocks, const StreamArgs &args,
                                  hipStream_t stream) {
    using namespace stream_detail;
    switch (U) {
        case 1: return dispatch_l<float, 4, 1>(L, blocks, args, stream);
        case 2: return dispatch_l<float, 4, 2>(L, blocks, args, stream);
        default: break;
    }
    return hipErrorInvalidValue;
}

}  // namespace pwa
