"""The build's barrier check: clean on the library, and it catches a kernel
whose barrier sits in a loop the compiler lowers as divergent.  Compiles to
assembly only; nothing runs on a GPU."""
import os
import textwrap

import pytest

from paper_0709_4552_amd import build, isa_check

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_0709_4552_amd", "csrc")


@pytest.mark.parametrize("name", ["kernels_force.hip", "kernels_step.hip"])
def test_library_kernels_have_no_divergent_barrier_loops(name, tmp_path):
    asm = build.device_asm(os.path.join(CSRC, name), str(tmp_path / (name + ".s")))
    assert isa_check.count_kernels(asm) > 0
    assert isa_check.check_asm(asm) == []


def test_check_catches_barrier_in_divergent_loop(tmp_path):
    # the loop's trip count comes from LDS per lane: the compiler must treat
    # the exit as divergent, with a barrier inside (never launched)
    src = tmp_path / "bad.hip"
    src.write_text(textwrap.dedent("""
        #include <hip/hip_runtime.h>
        __global__ void bad(int *out, const int *in) {
            __shared__ int cnt[256];
            cnt[threadIdx.x] = in[threadIdx.x];
            __syncthreads();
            int s = 0;
            for (int k = 0; k < cnt[threadIdx.x]; k++) {
                __syncthreads();
                s += cnt[(threadIdx.x + k) & 255];
            }
            out[threadIdx.x] = s;
        }
    """))
    asm = build.device_asm(str(src), str(tmp_path / "bad.s"))
    assert isa_check.check_asm(asm), "checker missed a barrier in a divergent loop"
