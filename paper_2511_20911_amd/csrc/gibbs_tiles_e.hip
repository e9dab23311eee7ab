// gibbs_tiles_e.hip -- compiled (L, R) variants of the Gibbs kernel, part e.
#include "gibbs_kernel.h"

namespace crbmlib {

#define TILE(l, r)                                              \
    if (L == l && R == r) {                                     \
        if (a) *err = gk::launch_tile<l, r>(*a, st);            \
        if (fn) *fn = gk::kernel_ptr<l, r>();                   \
        return true;                                            \
    }

bool tiles_e(int L, int R, const GibbsArgs* a, hipStream_t st, hipError_t* err,
             const void** fn) {
    TILE(48, 1)
    TILE(48, 2)
    TILE(48, 3)
    TILE(48, 4)
    TILE(48, 6)
    TILE(64, 1)
    TILE(64, 2)
    TILE(64, 4)
    return false;
}

}  // namespace crbmlib
