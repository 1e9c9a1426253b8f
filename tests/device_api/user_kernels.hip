// User kernels written against the public device headers only, as a library
// user would write them, with C launchers for the GPU tests.  They draw from
// the streams of a set created by the library (its state planes and jump
// tables) and are checked against the oracle.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mrg32k3a_device.h"
#include "philox_device.h"

// Thread i: substream i of stream `base` (i * 2^76 values ahead, sec. 4.1),
// then e more values, then one uint32, one binary32 and one binary64 draw.
template <class G>
__global__ void mrg_user_kernel(const uint32_t *planes, uint64_t n_streams, uint64_t base,
                                const uint32_t *tables, uint64_t e, uint64_t count, uint32_t *u,
                                float *f, double *d)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    mrg::Stream<G> s;
    s.load(planes, n_streams, base);
    s.substream(tables, i);
    s.jump(tables, e);
    const uint32_t a = s.next_u32();
    const float b = s.next_f32();
    const double c = s.next_f64();
    u[i] = a;
    f[i] = b;
    d[i] = c;
}

// Thread i: k uint32 draws of Philox stream i, a jump of e, one binary32 and
// one binary64 draw; the position is stored back.
__global__ void philox_user_kernel(uint32_t *planes, uint64_t n_streams, int k, uint64_t e,
                                   uint32_t *u, float *f, double *d)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_streams) return;
    mrg::PhiloxStream s;
    s.load(planes, n_streams, i);
    for (int j = 0; j < k; ++j) u[i * k + j] = s.next_u32();
    s.jump(e);
    const float b = s.next_f32();
    const double c = s.next_f64();
    f[i] = b;
    d[i] = c;
    s.store(planes, n_streams, i);
}

extern "C" int user_mrg_draws(const uint32_t *planes, uint64_t n_streams, uint64_t base,
                              const uint32_t *tables, uint64_t e, uint64_t count, int engine,
                              uint32_t *u, float *f, double *d)
{
    if (count == 0) return 0;
    const unsigned grid = (unsigned)((count + 255) / 256);
    if (engine == 0)
        hipLaunchKernelGGL(mrg_user_kernel<mrg::GenI>, dim3(grid), dim3(256), 0, 0, planes,
                           n_streams, base, tables, e, count, u, f, d);
    else
        hipLaunchKernelGGL(mrg_user_kernel<mrg::GenF>, dim3(grid), dim3(256), 0, 0, planes,
                           n_streams, base, tables, e, count, u, f, d);
    if (hipGetLastError() != hipSuccess) return 1;
    return hipDeviceSynchronize() == hipSuccess ? 0 : 2;
}

extern "C" int user_philox_draws(uint32_t *planes, uint64_t n_streams, int k, uint64_t e,
                                 uint32_t *u, float *f, double *d)
{
    if (n_streams == 0) return 0;
    const unsigned grid = (unsigned)((n_streams + 255) / 256);
    hipLaunchKernelGGL(philox_user_kernel, dim3(grid), dim3(256), 0, 0, planes, n_streams, k, e,
                       u, f, d);
    if (hipGetLastError() != hipSuccess) return 1;
    return hipDeviceSynchronize() == hipSuccess ? 0 : 2;
}
