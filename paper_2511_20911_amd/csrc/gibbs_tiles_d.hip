// gibbs_tiles_d.hip -- compiled (L, R) variants of the Gibbs kernel, part d.
#include "gibbs_kernel.h"

namespace crbmlib {

#define TILE(l, r)                                              \
    if (L == l && R == r) {                                     \
        if (a) *err = gk::launch_tile<l, r>(*a, st);            \
        if (fn) *fn = gk::kernel_ptr<l, r>();                   \
        return true;                                            \
    }

bool tiles_d(int L, int R, const GibbsArgs* a, hipStream_t st, hipError_t* err,
             const void** fn) {
    TILE(36, 1)
    TILE(36, 2)
    TILE(36, 3)
    TILE(36, 9)
    TILE(40, 1)
    TILE(40, 2)
    TILE(40, 4)
    TILE(40, 5)
    return false;
}

}  // namespace crbmlib
