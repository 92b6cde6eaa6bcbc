// Instantiations of the fused likelihood kernel for float amplitudes, 8 complex per lane.
#include "nll_stream_impl.hpp"

namespace pwa {

hipError_t stream_dispatch_f32_c8(int L, int U, int blocks, const StreamArgs &args,
                                  hipStream_t stream) {
    using namespace stream_detail;
    switch (U) {
        case 1: return dispatch_l<float, 8, 1>(L, blocks, args, stream);
        default: break;
    }
    return hipErrorInvalidValue;
}

}  // namespace pwa
