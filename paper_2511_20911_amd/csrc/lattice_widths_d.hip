// lattice_widths_d.hip -- general-lattice kernels compiled for column counts
// 50 .. 64, part d.
#include "lattice_kernel.h"

namespace crbmlib {
namespace lat {

#define WIDTH(lc)                                   \
    if (Lc == lc) {                                 \
        *err = launch_width<lc>(a, lds, st);        \
        return true;                                \
    }

bool widths_d(int Lc, const LatArgs& a, int lds, hipStream_t st, hipError_t* err) {
    WIDTH(50)
    WIDTH(52)
    WIDTH(54)
    WIDTH(56)
    WIDTH(58)
    WIDTH(60)
    WIDTH(62)
    WIDTH(64)
    return false;
}

}  // namespace lat
}  // namespace crbmlib
