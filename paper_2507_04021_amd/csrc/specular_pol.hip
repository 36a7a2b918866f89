// Instances of the refinement kernel with the polarised field (Jones
// vectors, PCRT_POLARIZED), in a translation unit of their own so that they
// compile in parallel with the scalar ones.
#include "refine.h"

namespace pcrt {

template <int W>
static void launch_pol_w(const LaunchArgs &A, dim3 grid, hipStream_t s) {
    if (A.rb.nk) launch_refine_wa<W, true, true>(A, grid, s);
    else launch_refine_wa<W, false, true>(A, grid, s);
}

void launch_refine_pol(const LaunchArgs &A, dim3 grid, hipStream_t s) {
    switch (A.D.width) {
        case 8: launch_pol_w<8>(A, grid, s); break;
        case 4: launch_pol_w<4>(A, grid, s); break;
        default: launch_pol_w<2>(A, grid, s); break;
    }
}

}  // namespace pcrt
