// lattice_widths_c.hip -- general-lattice kernels compiled for column counts
// 34 .. 48, part c.
#include "lattice_kernel.h"

namespace crbmlib {
namespace lat {

#define WIDTH(lc)                                   \
    if (Lc == lc) {                                 \
        *err = launch_width<lc>(a, lds, st);        \
        return true;                                \
    }

bool widths_c(int Lc, const LatArgs& a, int lds, hipStream_t st, hipError_t* err) {
    WIDTH(34)
    WIDTH(36)
    WIDTH(38)
    WIDTH(40)
    WIDTH(42)
    WIDTH(44)
    WIDTH(46)
    WIDTH(48)
    return false;
}

}  // namespace lat
}  // namespace crbmlib
