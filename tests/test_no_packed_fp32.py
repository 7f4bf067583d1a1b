"""Device code is built without packed FP32 arithmetic (v_pk_fma/mul/add_f32):
compile every HIP source to gfx950 assembly with the library's own flags and
scan it."""
import concurrent.futures as cf
import glob
import os
import re
import subprocess

from paper_2005_10494_amd import build as B


def _asm(src, outdir):
    out = os.path.join(outdir, os.path.basename(src) + ".s")
    subprocess.check_call([B.HIPCC, *B.CFLAGS, "--cuda-device-only", "-S", src, "-o", out],
                          stderr=subprocess.DEVNULL)
    with open(out) as f:
        return src, f.read()


def test_device_assembly_has_no_packed_fp32(tmp_path):
    srcs = sorted(glob.glob(os.path.join(B.CSRC, "*.hip")))
    assert srcs
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(lambda s: _asm(s, str(tmp_path)), srcs))
    for src, asm in results:
        assert "amdgcn" in asm
        bad = re.findall(r"\bv_pk_(?:fma|mul|add)_f32\b", asm)
        assert not bad, (src, bad[:3])
