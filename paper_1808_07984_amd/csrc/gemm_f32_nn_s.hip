// Instantiation of the fp32 Strassen kernels: A and B as stored, 128x128x32 tile.
#include "gemm_f32.hpp"

namespace strassen {

hipError_t launch_f32_nn_s(int wa, int wb, int wc, const LaunchArgs &a, int batch,
                                 bool vec, hipStream_t s) {
    return f32k::dispatch<f32k::Small, true, false>(wa, wb, wc, a, batch, vec, s);
}

hipError_t launch_f32_conc_s(int wmax, const LaunchArgs &a, int batch, bool vec, hipStream_t s) {
    return f32k::dispatch_concurrent<f32k::Small>(wmax, a, batch, vec, s);
}

}  // namespace strassen
