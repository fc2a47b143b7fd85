// Explicit instantiation of the SELBM kernels: dim 3, Q 19, storage float.
#include "launch_impl.h"

namespace sel {

const Ops *ops_d3q19_fp32(int N)
{
    switch (N) {
    case 2: return Impl<3, 2, 19, float, true>::ops();
    case 3: return Impl<3, 3, 19, float, true>::ops();
    case 4: return Impl<3, 4, 19, float, true>::ops();
    case 5: return Impl<3, 5, 19, float, true>::ops();
    case 6: return Impl<3, 6, 19, float, true>::ops();
    case 7: return Impl<3, 7, 19, float, true>::ops();
    case 8: return Impl<3, 8, 19, float, true>::ops();
    // the Taylor-Green order of Sec. 3.4 (several nodes per thread)
    case 12: return Impl<3, 12, 19, float, true>::ops();
    default: return nullptr;
    }
}

}  // namespace sel
