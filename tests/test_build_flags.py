"""Build-flag checks that need no GPU: the device code keeps binary16
denormals.  The 16-bit integer cells are ordered with a binary16 maximum
(pmax3 in the kernels), which is exact only if subnormal binary16 values
(the cell values 1..1023) are not flushed to zero; the library's build flags
pin IEEE denormal handling, and this test compiles a kernel that uses the
same packed maximum with those flags and reads the mode the compiler wrote
into its kernel descriptor."""
import os
import shutil
import subprocess
import tempfile

import pytest

from paper_2301_09310_amd import build as B

PROBE = r'''
#include <hip/hip_runtime.h>
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
__global__ void probe(unsigned *out, unsigned a, unsigned b, unsigned c) {
    const f16x2 x = __builtin_bit_cast(f16x2, a), y = __builtin_bit_cast(f16x2, b),
                z = __builtin_bit_cast(f16x2, c);
    out[threadIdx.x] = __builtin_bit_cast(unsigned, __builtin_elementwise_maximum(
        __builtin_elementwise_maximum(x, y), z));
}
'''


@pytest.mark.skipif(not os.path.exists(B.HIPCC), reason="hipcc not installed")
def test_device_code_keeps_f16_denormals():
    assert "-fdenormal-fp-math=ieee" in B.DEVICE
    tmp = tempfile.mkdtemp(prefix="salo_flags_")
    try:
        src = os.path.join(tmp, "probe.hip")
        with open(src, "w") as f:
            f.write(PROBE)
        out = os.path.join(tmp, "probe.s")
        cmd = [B.HIPCC] + B.COMMON + B.DEVICE + ["--offload-device-only", "-S", "-x", "hip",
                                                  src, "-o", out]
        subprocess.run(cmd, check=True, capture_output=True)
        asm = open(out).read()
        modes = [line.split()[-1] for line in asm.splitlines()
                 if ".amdhsa_float_denorm_mode_16_64" in line]
        assert modes and all(m == "3" for m in modes), modes   # 3: keep input and output denormals
        assert "v_pk_maximum3_f16" in asm or "v_pk_max" in asm
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
