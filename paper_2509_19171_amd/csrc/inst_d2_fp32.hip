// Explicit instantiation of the SELBM kernels: dim 2, Q 9, storage float.
#include "launch_impl.h"

namespace sel {

const Ops *ops_d2_fp32(int N)
{
    switch (N) {
    case 2: return Impl<2, 2, 9, float, true>::ops();
    case 3: return Impl<2, 3, 9, float, true>::ops();
    case 4: return Impl<2, 4, 9, float, true>::ops();
    case 5: return Impl<2, 5, 9, float, true>::ops();
    case 6: return Impl<2, 6, 9, float, true>::ops();
    case 7: return Impl<2, 7, 9, float, true>::ops();
    case 8: return Impl<2, 8, 9, float, true>::ops();
    case 9: return Impl<2, 9, 9, float, true>::ops();
    case 10: return Impl<2, 10, 9, float, true>::ops();
    default: return nullptr;
    }
}

}  // namespace sel
