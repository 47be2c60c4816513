"""The HIP kernels are compiled without packed FP32 instructions and with the exactness
flags the numerical definition relies on (checked on the generated gfx950 assembly)."""
import os
import re
import shutil
import subprocess

import pytest

from paper_2210_06160_amd import build

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc missing")


@pytest.mark.parametrize("src", [s for s in build.SOURCES if s.endswith(".hip")])
def test_no_packed_fp32(src, tmp_path):
    out = tmp_path / (src + ".s")
    cmd = ["hipcc", *build.FLAGS, "-x", "hip", "-S", "--cuda-device-only",
           os.path.join(build.CSRC, src), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    asm = out.read_text()
    bad = re.findall(r"\bv_pk_(?:add|mul|fma)_f32\b", asm)
    assert not bad, "%s uses packed FP32: %s" % (src, sorted(set(bad)))


def test_exactness_flags():
    for f in ("-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt",
              "-fno-gpu-flush-denormals-to-zero", "-packed-fp32-ops"):
        assert f in build.FLAGS
