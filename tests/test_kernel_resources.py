"""The HIP kernels' resource use, read from the gfx950 code object the build
makes (no GPU needed): no kernel spills to scratch memory, and the
single-lattice bond kernels keep the register budget of their occupancy."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1202_0635_amd", "csrc")


@pytest.fixture(scope="module")
def kernels(tmp_path_factory):
    from paper_1202_0635_amd import build

    out = str(tmp_path_factory.mktemp("isa") / "sw_kernels.s")
    cmd = [build.hipcc(), *[f for f in build.HIPCC_FLAGS if f not in ("-fPIC", "-shared", "-Wall")],
           "--cuda-device-only", "-S", "-I", build.INCLUDE, "-I", CSRC,
           os.path.join(CSRC, "sw_kernels.hip"), "-o", out]
    try:
        subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    except FileNotFoundError:
        pytest.skip("hipcc not available")
    text = open(out).read()
    res = {}
    for m in re.finditer(r"\.amdhsa_kernel (\S+)(.*?)\.end_amdhsa_kernel", text, flags=re.S):
        body = m.group(2)
        field = lambda k: int(re.search(rf"\.amdhsa_{k} (\d+)", body).group(1))
        res[m.group(1)] = {"scratch": field("private_segment_fixed_size"), "vgpr": field("next_free_vgpr"),
                           "lds": field("group_segment_fixed_size")}
    assert res, "no kernels found in the code object"
    return res


def test_no_kernel_spills_to_scratch(kernels):
    spilled = {k: v["scratch"] for k, v in kernels.items() if v["scratch"]}
    assert not spilled, spilled


def test_code_kernels_keep_their_occupancy(kernels):
    # the single-lattice bond kernels (two-level labels): Potts within the
    # register budget of eight waves per SIMD, the clock model within seven
    code = {k: v for k, v in kernels.items() if "k_code_bond" in k}
    assert len(code) == 8  # Potts and clock, from spins or codes, 4 and 8 waves per tile
    for k, v in code.items():
        waves = 7 if "clock" in k else 8
        assert v["vgpr"] <= 512 // waves, (k, v)
        assert waves * v["lds"] <= 160 * 1024, (k, v)
