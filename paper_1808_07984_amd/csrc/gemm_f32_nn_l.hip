// Instantiation of the fp32 Strassen kernels: A and B as stored, 256x256x16 tile.
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
