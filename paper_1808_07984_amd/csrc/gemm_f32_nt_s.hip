// Instantiation of the fp32 Strassen kernels: A as stored, B transposed, 128x128x32 tile.
#include "gemm_f32.hpp"

namespace strassen {

hipError_t launch_f32_nt_s(int wa, int wb, int wc, const LaunchArgs &a, int batch,
                                 bool vec, hipStream_t s) {
    return f32k::dispatch<f32k::Small, true, true>(wa, wb, wc, a, batch, vec, s);
}

}  // namespace strassen
