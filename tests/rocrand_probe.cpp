// Test helper: one Philox4x32-10 block computed by rocRAND's own engine
// (host side), used as an external reference for the oracle's and the
// kernels' Philox.  rocRAND is called as a library; nothing is copied.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <stdint.h>

extern "C" void rocrand_philox_block(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
    const unsigned long long seed = (unsigned long long)key[0] | ((unsigned long long)key[1] << 32);
    const unsigned long long subsequence = (unsigned long long)ctr[2] | ((unsigned long long)ctr[3] << 32);
    const unsigned long long offset = 4ull * ((unsigned long long)ctr[0] | ((unsigned long long)ctr[1] << 32));
    rocrand_device::philox4x32_10_engine eng(seed, subsequence, offset);
    const uint4 r = eng.next4();
    out[0] = r.x;
    out[1] = r.y;
    out[2] = r.z;
    out[3] = r.w;
}
