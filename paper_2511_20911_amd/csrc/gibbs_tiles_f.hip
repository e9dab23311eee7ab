// gibbs_tiles_f.hip -- compiled (L, R) variants of the Gibbs kernel, part f.
#include "gibbs_kernel.h"

namespace crbmlib {

#define TILE(l, r)                                              \
    if (L == l && R == r) {                                     \
        if (a) *err = gk::launch_tile<l, r>(*a, st);            \
        if (fn) *fn = gk::kernel_ptr<l, r>();                   \
        return true;                                            \
    }

bool tiles_f(int L, int R, const GibbsArgs* a, hipStream_t st, hipError_t* err,
             const void** fn) {
    TILE(72, 1)
    TILE(72, 2)
    TILE(72, 3)
    TILE(72, 4)
    TILE(96, 1)
    TILE(96, 2)
    TILE(96, 3)
    TILE(96, 4)
    return false;
}

}  // namespace crbmlib
