// Host-side wrapper around rocRAND's Philox4x32-10 engine, used by the test
// suite as an independent implementation to check the oracle's Philox.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdint>

extern "C" void rr_philox_next4(unsigned long long seed, unsigned long long subsequence,
                                unsigned long long offset, uint32_t* out)
{
    rocrand_device::philox4x32_10_engine eng(seed, subsequence, offset);
    uint4 r = eng.next4();
    out[0] = r.x; out[1] = r.y; out[2] = r.z; out[3] = r.w;
}
