"""Write the 128^3, chi = 128 velocity fixture from the CPU FP64 MPS oracle.

The fixture is the reference of the GPU parity test of the branching-tube
configuration at full size (128^3 grid, chi = 128, tol 1e-8, tau 0.55,
velocity inlet 0.02, pressure outlet, obstacle mask at machine
precision): the oracle (oracle/mps_lbm.py, the step of Section 3.2 on MPS
populations) runs two steps from the seeded flow the test also starts from,
and the velocity u = j / rho of its final populations is stored at a seeded
sample of fluid cells.  Only oracle/ and the input generators are used.

    python tests/golden/make_vascular128_fixture.py [out.txt]

Takes tens of minutes on a few CPU cores.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as WL  # noqa: E402
from oracle.dense_lbm import moments  # noqa: E402
from oracle.mps_lbm import MPSLBM  # noqa: E402

SAMPLES = 6000
SAMPLE_SEED = 2515


def case():
    c = WL.case_vascular(n=7, chi=128, tau=0.55, tol=1e-8)
    rho, u = WL.random_flow_state(c.n, 3, amp=0.01)
    c.rho_init, c.u_init = rho, u
    return c


def sample_cells(solid):
    fluid = np.argwhere(solid == 0)
    rng = np.random.default_rng(SAMPLE_SEED)
    pick = np.sort(rng.choice(len(fluid), size=SAMPLES, replace=False))
    return fluid[pick]


def main(out):
    c = case()
    t0 = time.time()
    m = MPSLBM(c)
    print(f"oracle initialised in {time.time() - t0:.0f} s, mask bonds "
          f"{[x.shape[2] for x in m.mask[:-1]]}", flush=True)
    for s in range(2):
        t1 = time.time()
        m.step()
        print(f"step {s + 1} in {time.time() - t1:.0f} s", flush=True)
    f = m.dense_populations()
    rho, j = moments(f)
    cells = sample_cells(c.solid)
    x, y, z = cells.T
    u = j[:, x, y, z] / rho[x, y, z]
    with open(out, "w") as fh:
        fh.write("# Velocity u = j / rho after two steps of the CPU FP64 MPS oracle\n")
        fh.write("# (Section 3.2 step on MPS populations) on the 128^3 branching-tube\n")
        fh.write("# configuration: chi 128, tol 1e-8, tau 0.55, velocity inlet (0.02,0,0)\n")
        fh.write("# on x = 0, pressure outlet rho_b = 1 on x = 127, obstacle mask at\n")
        fh.write("# machine precision, Taylor-2 inverse density, two sweeps per product;\n")
        fh.write("# start: workloads.random_flow_state(7, seed 3, amp 0.01).\n")
        fh.write(f"# {SAMPLES} fluid cells drawn with numpy default_rng({SAMPLE_SEED}).\n")
        fh.write(f"# oracle mass {m.mass():.17e}\n")
        fh.write(f"# rms |u| over the sample {float(np.sqrt((u ** 2).sum(0).mean())):.6e}\n")
        fh.write("# x y z ux uy uz\n")
        for k in range(SAMPLES):
            fh.write(f"{x[k]} {y[k]} {z[k]} {u[0, k]:.17e} {u[1, k]:.17e} {u[2, k]:.17e}\n")
    print("wrote", out, flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else
         os.path.join(os.path.dirname(os.path.abspath(__file__)),
                      "vascular128_chi128_velocity_samples.txt"))
