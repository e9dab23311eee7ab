// gibbs_tiles_c.hip -- compiled (L, R) variants of the Gibbs kernel, part c.
#include "gibbs_kernel.h"

namespace crbmlib {

#define TILE(l, r)                                              \
    if (L == l && R == r) {                                     \
        if (a) *err = gk::launch_tile<l, r>(*a, st);            \
        if (fn) *fn = gk::kernel_ptr<l, r>();                   \
        return true;                                            \
    }

bool tiles_c(int L, int R, const GibbsArgs* a, hipStream_t st, hipError_t* err,
             const void** fn) {
    TILE(28, 1)
    TILE(28, 2)
    TILE(28, 7)
    TILE(30, 1)
    TILE(30, 3)
    TILE(30, 5)
    TILE(32, 1)
    TILE(32, 2)
    TILE(32, 4)
    TILE(32, 8)
    return false;
}

}  // namespace crbmlib
