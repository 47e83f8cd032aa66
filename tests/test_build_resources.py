"""Register and scratch budget of the fast cell kernels, read from the compiler's
resource report (hipcc for gfx950, the library's own flags; no GPU needed).

A captured reference or a dynamically indexed register array silently moves state to
per-lane scratch memory, which costs the VALU-bound cell kernel a large share of its
speed; this test fails if that happens again."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _resources(src="cells.hip"):
    from paper_2601_05765_amd import build as b
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    out = os.path.join(ROOT, "_build", "resource_check_" + src.replace(".", "_") + ".o")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    cmd = [hipcc, *b.CFLAGS, "-x", "hip", "-c", os.path.join(b.CSRC, src), "-o", out,
           "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    res, cur = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            res[cur] = {}
            continue
        m = re.search(r"(VGPRs|ScratchSize \[bytes/lane\]): (\d+)", line)
        if m and cur:
            res[cur][m.group(1).split()[0]] = int(m.group(2))
    return res


def test_fast_cell_kernels_use_no_scratch():
    res = _resources()
    fast = {k: v for k, v in res.items() if "k_cells_fast" in k}
    assert len(fast) >= 5, sorted(res)
    for name, v in fast.items():
        assert v.get("ScratchSize") == 0, (name, v)
    # 32 lanes per cell (the default): at most 96 VGPRs, i.e. at least 5 waves per SIMD
    main = [v for k, v in fast.items() if "ILi32ELb0E" in k]
    assert main and main[0]["VGPRs"] <= 96, fast


def test_fluid_kernels_use_no_scratch():
    """The fluid model's row kernel and the three-coordinate PCG keep their state in
    registers (the PCG iteration runs ~65 times per velocity update)."""
    res = _resources("fluid.hip")
    names = [k for k in res if any(t in k for t in ("k_cg3_iter", "k_cg3_init", "k_fluid_rows", "k_p1_laplacian"))]
    assert len(names) == 4, sorted(res)
    for name in names:
        assert res[name].get("ScratchSize") == 0, (name, res[name])
