"""Write the FP64 oracle gradient of the strain-squared loss for the adjoint recipe on 16^3
(500 steps, checkpoint every 50) to adjoint_c4_16cubed_500.npz.

Calls only oracle/ and synth/: seeded spectrum velocity (seed 1704, u_rms 0.04), force
field U(-1e-6, 1e-6) (seed 7559), rho0 = 1, tau_nu = 0.8, d'Humieres rates.

    python tests/golden/make_adjoint_golden.py
"""
import sys
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

import synth  # noqa: E402
from oracle import adjoint as adj  # noqa: E402
from oracle import d3q19 as d  # noqa: E402

N, STEPS, EVERY = 16, 500, 50


def main():
    shape = (N, N, N)
    u0 = synth.spectrum_velocity(shape, seed=1704, u_rms=0.04)
    F = synth.uniform_random_force(shape, seed=7559, amp=1e-6)
    p = d.Params(s=d.default_rates(0.8))
    J, gu, gF = adj.gradient(u0, F, p, STEPS, every=EVERY)
    out = Path(__file__).with_name("adjoint_c4_16cubed_500.npz")
    np.savez_compressed(out, J=np.array(J), grad_u0=gu, grad_F=gF, steps=STEPS, every=EVERY)
    print(f"J = {J:.17g}; wrote {out}")


if __name__ == "__main__":
    main()
