// Instantiations of the fused likelihood kernel for float amplitudes, 1 complex per lane.
#include "nll_stream_impl.hpp"

namespace pwa {

hipError_t stream_dispatch_f32_c1(int L, int U, int blocks, const StreamArgs &args,
                                  hipStream_t stream) {
    using namespace stream_detail;
    switch (U) {
        case 4: return dispatch_l<float, 1, 4>(L, blocks, args, stream);
        case 8: return dispatch_l<float, 1, 8>(L, blocks, args, stream);
        default: break;
    }
    return hipErrorInvalidValue;
}

}  // namespace pwa
