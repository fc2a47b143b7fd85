// Explicit instantiation of the SELBM kernels: dim 3, Q 27, storage double.
#include "launch_impl.h"

namespace sel {

const Ops *ops_d3q27_fp64(int N)
{
    switch (N) {
    case 2: return Impl<3, 2, 27, double, false>::ops();
    case 3: return Impl<3, 3, 27, double, false>::ops();
    case 4: return Impl<3, 4, 27, double, false>::ops();
    case 5: return Impl<3, 5, 27, double, false>::ops();
    case 6: return Impl<3, 6, 27, double, false>::ops();
    case 7: return Impl<3, 7, 27, double, false>::ops();
    case 8: return Impl<3, 8, 27, double, false>::ops();
    default: return nullptr;
    }
}

}  // namespace sel
