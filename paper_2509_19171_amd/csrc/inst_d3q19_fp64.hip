// Explicit instantiation of the SELBM kernels: dim 3, Q 19, storage double.
#include "launch_impl.h"

namespace sel {

const Ops *ops_d3q19_fp64(int N)
{
    switch (N) {
    case 2: return Impl<3, 2, 19, double, false>::ops();
    case 3: return Impl<3, 3, 19, double, false>::ops();
    case 4: return Impl<3, 4, 19, double, false>::ops();
    case 5: return Impl<3, 5, 19, double, false>::ops();
    case 6: return Impl<3, 6, 19, double, false>::ops();
    case 7: return Impl<3, 7, 19, double, false>::ops();
    case 8: return Impl<3, 8, 19, double, false>::ops();
    // the Taylor-Green order of Sec. 3.4 (several nodes per thread)
    case 12: return Impl<3, 12, 19, double, false>::ops();
    default: return nullptr;
    }
}

}  // namespace sel
