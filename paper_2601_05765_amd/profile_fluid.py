#!/usr/bin/env python3
"""A short run of the fluid model's velocity update for kernel-trace profiles.

Solves the dam-break workload (100,000 sites) once, then calls lagot_fluid_velocity
five times at the converged weights (random velocities, per-site viscosity in [0, 2],
m = nu, dt = 2e-3, eps = 0.02, gamma = 0.05), as the bench's fluid section does.

    rocprofv3 --kernel-trace --stats -d OUT -o fluid -- python3 paper_2601_05765_amd/profile_fluid.py
"""
from __future__ import annotations

import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


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
    st = ctx.solve(x, y, z, nu, psi, opts=L.default_opts(tol=1e-5))
    print(f"profile_fluid: solve of dam_break {n}: status {st.status}", flush=True)
    g = torch.Generator(device="cuda").manual_seed(3)
    v = torch.randn((n, 3), generator=g, dtype=torch.float64, device="cuda")
    mu = 2.0 * torch.rand(n, generator=g, dtype=torch.float64, device="cuda")
    prm = L.default_fluid_params(dt=2e-3, eps=0.02, gamma=0.05)
    for k in range(5):
        _, _, its = ctx.fluid_velocity(x, y, z, psi, nu, v, prm, mu=mu)
        print(f"profile_fluid: velocity update {k}: PCG iterations {its}", flush=True)
    torch.cuda.synchronize()
    return 0


if __name__ == "__main__":
    sys.exit(main())
