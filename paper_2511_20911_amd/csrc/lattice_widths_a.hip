// lattice_widths_a.hip -- general-lattice kernels compiled for column counts
// 4 .. 16, part a.
#include "lattice_kernel.h"

namespace crbmlib {
namespace lat {

#define WIDTH(lc)                                   \
    if (Lc == lc) {                                 \
        *err = launch_width<lc>(a, lds, st);        \
        return true;                                \
    }

bool widths_a(int Lc, const LatArgs& a, int lds, hipStream_t st, hipError_t* err) {
    WIDTH(4)
    WIDTH(6)
    WIDTH(8)
    WIDTH(10)
    WIDTH(12)
    WIDTH(14)
    WIDTH(16)
    return false;
}

}  // namespace lat
}  // namespace crbmlib
