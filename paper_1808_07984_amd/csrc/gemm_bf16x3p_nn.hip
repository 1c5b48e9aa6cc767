// Instantiation of the 16-bit MFMA Strassen kernels in the compensated bf16x3
// mode on pre-split operands (A pre-split, B pre-split or fp32), A and B as
// stored: the single-term products of the formed one-level schedule.
#include "gemm_mfma16.hpp"

namespace strassen {

hipError_t launch_m16_x3pre(bool pre_b, bool large, int wa, int wb, int wc, const LaunchArgs &a, int batch,
                            bool vec, hipStream_t s) {
    using Both = m16k::X3PreOps<true, true>;
    using AOnly = m16k::X3PreOps<true, false>;
    if (pre_b)
        return large ? m16k::dispatch_pre<m16k::LargeX3, Both>(wa, wb, wc, a, batch, vec, s)
                     : m16k::dispatch_pre<m16k::Small, Both>(wa, wb, wc, a, batch, vec, s);
    return large ? m16k::dispatch_pre<m16k::LargeX3, AOnly>(wa, wb, wc, a, batch, vec, s)
                 : m16k::dispatch_pre<m16k::Small, AOnly>(wa, wb, wc, a, batch, vec, s);
}

hipError_t launch_m16_x3pre_chained(const LaunchArgs &a, int nchains, bool vec, hipStream_t s) {
    using Both = m16k::X3PreOps<true, true>;
    return m16k::launch_chained<m16k::TileFor<m16k::LargeX3, Both, 1, 1, true, false>, Both>(a, nchains, vec, s);
}

}  // namespace strassen
