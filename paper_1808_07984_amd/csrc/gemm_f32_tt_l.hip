// Instantiation of the fp32 Strassen kernels: A and B transposed, 256x256x16 tile.
#include "gemm_f32.hpp"

namespace strassen {

hipError_t launch_f32_tt_l(int wa, int wb, int wc, const LaunchArgs &a, int batch,
                                 bool vec, hipStream_t s) {
    return f32k::dispatch<f32k::Large, false, true>(wa, wb, wc, a, batch, vec, s);
}

}  // namespace strassen
