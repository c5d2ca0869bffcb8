// Test helper: exposes rocRAND's own Philox4x32-10 round function (a library
// implementation independent of the oracle) through a C symbol.  Built host-only.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdint>

namespace {
struct Engine : rocrand_device::philox4x32_10_engine {
    uint4 rounds(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
}  // namespace

extern "C" void rocrand_philox_ref(const uint32_t* ctr, const uint32_t* key, uint32_t* out)
{
    Engine e;
    uint4 c;
    c.x = ctr[0];
    c.y = ctr[1];
    c.z = ctr[2];
    c.w = ctr[3];
    uint2 k;
    k.x = key[0];
    k.y = key[1];
    const uint4 r = e.rounds(c, k);
    out[0] = r.x;
    out[1] = r.y;
    out[2] = r.z;
    out[3] = r.w;
}
