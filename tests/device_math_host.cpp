// Host build of the kernels' range-specialised elementary functions
// (log_unit, cos2_turn, sincos_turn from device_math.h), evaluated on the
// uniforms (r + 1) / 2^32 for the 32-bit words r read from stdin; writes one
// line of results per word.  Built and checked by test_device_math_host.py.
#include <cstdio>
#include <cstdint>

#include "device_math.h"

int main()
{
    unsigned long long r;
    while (std::scanf("%llu", &r) == 1) {
        const double u = su3hb::u01(uint32_t(r));
        double sd, cd;
        float sf, cf;
        su3hb::sincos_turn<double>(u, &sd, &cd);
        su3hb::sincos_turn<float>(u, &sf, &cf);
        std::printf("%a %a %a %a %a %a\n", su3hb::log_unit(u, su3hb::kLogTable), su3hb::cos2_turn(u), sd, cd, double(sf), double(cf));
    }
    return 0;
}
