"""The public device headers (include/mrg32k3a_device.h, include/philox_device.h)
are self-contained: user kernels that include only them compile for gfx950
(compile only, no GPU).  tests/test_gpu_device_api.py runs such user kernels
on the GPU against the oracle."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"

USER_KERNEL = r"""
#include "mrg32k3a_device.h"

// Each thread sums k uniforms of its own stream and continues it next launch.
__global__ void mean_kernel(uint32_t *planes, uint64_t n_streams, int k, float *out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_streams) return;
    mrg::Stream<> s;
    s.load(planes, n_streams, i);
    float acc = 0.f;
    for (int j = 0; j < k; ++j) acc += s.next_f32();
    s.store(planes, n_streams, i);
    out[i] = acc / k;
}

// Thread i draws from substream i of stream 0, then jumps 1000 values.
__global__ void int_kernel(const uint32_t *planes, uint64_t n_streams, const uint32_t *tables,
                           uint32_t *out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_streams) return;
    mrg::Stream<mrg::GenI> s;
    s.load(planes, n_streams, 0);
    s.substream(tables, i);
    s.jump(tables, 1000);
    out[i] = s.next_u32();
    out[n_streams + i] = (uint32_t)(s.next_f64() * 4294967296.0);
}
"""


PHILOX_KERNEL = r"""
#include "philox_device.h"

// Each thread draws k values of its Philox stream, skips 2^40, draws one more.
__global__ void philox_user(uint32_t *planes, uint64_t n_streams, int k, double *out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_streams) return;
    mrg::PhiloxStream s;
    s.load(planes, n_streams, i);
    double acc = 0.0;
    for (int j = 0; j < k; ++j) acc += s.next_f64() + s.next_f32() + (double)s.next_u32();
    s.jump((uint64_t)1 << 40);
    out[i] = acc + s.next_f64();
    s.store(planes, n_streams, i);
}
"""


def compile_device(tmp_path, name, text):
    src = tmp_path / (name + ".hip")
    src.write_text(text)
    out = tmp_path / (name + ".o")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "--offload-device-only", "-O3",
                           "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                           "-packed-fp32-ops", "-Wno-unused-command-line-argument",
                           "-I", os.path.join(ROOT, "include"), "-c", str(src), "-o", str(out)],
                          stderr=subprocess.DEVNULL)
    return out


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="no hipcc")
def test_philox_user_kernel_compiles_with_public_header(tmp_path):
    assert compile_device(tmp_path, "philox_user", PHILOX_KERNEL).stat().st_size > 0


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="no hipcc")
def test_user_kernel_compiles_with_public_header(tmp_path):
    src = tmp_path / "user.hip"
    src.write_text(USER_KERNEL)
    out = tmp_path / "user.o"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "--offload-device-only", "-O3",
                           "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                           "-packed-fp32-ops", "-Wno-unused-command-line-argument",
                           "-I", os.path.join(ROOT, "include"), "-c", str(src), "-o", str(out)],
                          stderr=subprocess.DEVNULL)
    assert out.stat().st_size > 0
