// Instantiation of the fp32 Strassen kernels: A and B as stored, 256x256 tile
// (32-deep k-tiles; 16-deep for variants with more than four operand terms
// other than (4,1,4) and (4,2,2)).
#include "gemm_f32.hpp"

namespace strassen {

hipError_t launch_f32_nn_l(int wa, int wb, int wc, const LaunchArgs &a, int batch,
                                 bool vec, hipStream_t s) {
    return f32k::dispatch<f32k::Large, true, false>(wa, wb, wc, a, batch, vec, s);
}

hipError_t launch_f32_conc_l(int wmax, const LaunchArgs &a, int batch, bool vec, hipStream_t s) {
    return f32k::dispatch_concurrent<f32k::Large>(wmax, a, batch, vec, s);
}

}  // namespace strassen
