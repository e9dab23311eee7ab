// lattice_widths_b.hip -- general-lattice kernels compiled for column counts
// 18 .. 32, part b.
#include "lattice_kernel.h"

namespace crbmlib {
namespace lat {

#define WIDTH(lc)                                   \
    if (Lc == lc) {                                 \
        *err = launch_width<lc>(a, lds, st);        \
        return true;                                \
    }

bool widths_b(int Lc, const LatArgs& a, int lds, hipStream_t st, hipError_t* err) {
    WIDTH(18)
    WIDTH(20)
    WIDTH(22)
    WIDTH(24)
    WIDTH(26)
    WIDTH(28)
    WIDTH(30)
    WIDTH(32)
    return false;
}

}  // namespace lat
}  // namespace crbmlib
