// Host-side selection among the fp32 kernel instantiations.
#include "launch.hpp"

namespace strassen {

KernelShape f32_tile_shape(bool large, int wa, int wb, int wc, bool untransposed) {
    // k-tile by operand terms: the large tile stages 16 deep above four terms
    // in all, except (4,1,4) and (4,2,2) with untransposed operands (32 deep,
    // split staging), and 32 deep otherwise
    const bool split = untransposed && wa == 4 && ((wb == 1 && wc == 4) || (wb == 2 && wc == 2));
    return large ? KernelShape{256, 256, wa + wb > 4 && !split ? 16 : 32, 4} : KernelShape{128, 128, 32, 4};
}

hipError_t launch_f32(bool trans_a, bool trans_b, bool large, int wa, int wb, int wc,
                      const LaunchArgs &a, int batch, bool vec, hipStream_t s) {
    if (!trans_a && !trans_b)
        return large ? launch_f32_nn_l(wa, wb, wc, a, batch, vec, s)
                     : launch_f32_nn_s(wa, wb, wc, a, batch, vec, s);
    if (!trans_a && trans_b)
        return large ? launch_f32_nt_l(wa, wb, wc, a, batch, vec, s)
                     : launch_f32_nt_s(wa, wb, wc, a, batch, vec, s);
    if (trans_a && !trans_b)
        return large ? launch_f32_tn_l(wa, wb, wc, a, batch, vec, s)
                     : launch_f32_tn_s(wa, wb, wc, a, batch, vec, s);
    return large ? launch_f32_tt_l(wa, wb, wc, a, batch, vec, s)
                 : launch_f32_tt_s(wa, wb, wc, a, batch, vec, s);
}

const char *f32_kernel_name(bool large) {
    return large ? "strassen_f32_kernel<256x256>" : "strassen_f32_kernel<128x128>";
}

}  // namespace strassen
