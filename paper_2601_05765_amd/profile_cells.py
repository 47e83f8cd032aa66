#!/usr/bin/env python3
"""A short run of the measured workload for hardware-counter profiles.

Runs one plain OT solve of the dam-break workload (100,000 sites, the solve that
bench.py times) and then a plain 256 MiB device-to-device copy. Under
``rocprofv3 --pmc FETCH_SIZE`` (and, in a second run, ``WRITE_SIZE``) the copy gives
the counter's reading for a known number of bytes (256 MiB read, 256 MiB written),
which scales the cell kernel's readings to bytes.

    rocprofv3 --pmc FETCH_SIZE -d OUT -o pmc -- python3 paper_2601_05765_amd/profile_cells.py
"""
from __future__ import annotations

import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

COPY_BYTES = 256 * 1024 * 1024


def main() -> int:
    import numpy as np
    import torch

    import paper_2601_05765_amd as L
    from paper_2601_05765_amd import scenes

    n = int(sys.argv[1]) if len(sys.argv) > 1 else 100_000
    sc = scenes.dam_break(n, 0)
    t = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    x, y, z, nu = t(sc.x, torch.float32), t(sc.y, torch.float32), t(sc.z, torch.float32), t(sc.nu, torch.float64)
    psi = t(sc.psi0, torch.float64)
    ctx = L.Context()
    ctx.set_threads_per_cell(32)
    print(f"profile_cells: solve of dam_break {n}", flush=True)
    st = ctx.solve(x, y, z, nu, psi, opts=L.default_opts(tol=1e-5))
    torch.cuda.synchronize()
    print(f"profile_cells: {st.evals} evaluations, status {st.status}", flush=True)
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"profile_cells: copy of {COPY_BYTES} bytes done", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
