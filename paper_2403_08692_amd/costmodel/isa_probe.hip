// isa_probe.hip -- one kernel per arithmetic building block of the shower,
// compiled for gfx950 only to read its instruction count from the assembly
// (isa_costs.py).  Never launched.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../csrc/vsh_device.hpp"
#include "../csrc/vsh_math.hpp"

using namespace vsh;

#define PROBE_D(name, expr)                                                      \
  extern "C" __global__ void probe_##name(const double* __restrict__ a,         \
                                          double* __restrict__ o) {              \
    const double x = a[threadIdx.x];                                             \
    const double y = a[threadIdx.x + 64];                                        \
    (void)y;                                                                     \
    o[threadIdx.x] = (expr);                                                     \
  }

PROBE_D(base, x)
PROBE_D(add, x + y)
PROBE_D(log, log(x))
PROBE_D(log_fast, log_series(x))
PROBE_D(exp, exp(x))
PROBE_D(pow, pow(x, y))
PROBE_D(sqrt, sqrt(x))
PROBE_D(div, x / y)
PROBE_D(log10, log10(x))
PROBE_D(sin, sin(x))
PROBE_D(cos, cos(x))

extern "C" __global__ void probe_sincos(const double* __restrict__ a, double* __restrict__ o) {
  double s, c;
  sincos(a[threadIdx.x], &s, &c);
  o[threadIdx.x] = s;
  o[threadIdx.x + 64] = c;
}

extern "C" __global__ void probe_philox(const uint32_t* __restrict__ a, uint32_t* __restrict__ o) {
  const U4 r = philox10(a[threadIdx.x], a[threadIdx.x + 64], a[threadIdx.x + 128], a[threadIdx.x + 192],
                        a[256], a[257]);
  o[threadIdx.x] = r.x;
  o[threadIdx.x + 64] = r.y;
  o[threadIdx.x + 128] = r.z;
  o[threadIdx.x + 192] = r.w;
}

extern "C" __global__ void probe_philox_base(const uint32_t* __restrict__ a, uint32_t* __restrict__ o) {
  o[threadIdx.x] = a[threadIdx.x];
  o[threadIdx.x + 64] = a[threadIdx.x + 64];
  o[threadIdx.x + 128] = a[threadIdx.x + 128];
  o[threadIdx.x + 192] = a[threadIdx.x + 192] ^ a[256] ^ a[257];
}

extern "C" __global__ void probe_unit(const uint32_t* __restrict__ a, double* __restrict__ o) {
  o[threadIdx.x] = unit(a[threadIdx.x], a[threadIdx.x + 64]);
}

extern "C" __global__ void probe_unit_base(const uint32_t* __restrict__ a, double* __restrict__ o) {
  o[threadIdx.x] = __hiloint2double((int)a[threadIdx.x], (int)a[threadIdx.x + 64]);  // the words' bits, stored
}
