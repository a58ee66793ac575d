"""Write the FP64 oracle's scalar flux at t = 1 for the 400 x 400 line source with
16 x 32 = 512 ordinates and sigma_as in {0, 1, 5} (beta 4.5, sigma_s 1, sigma_a 0,
CFL 0.95 on the streaming, 197 forward-Euler steps).

Only the oracle and the seeded input description run here; nothing from the
GPU library.  Output: line_source_400_q512_phi.npz with one float32 [400, 400]
array per sigma_as (phi_as0, phi_as1, phi_as5) plus the oracle's step count and
dt; float32 storage keeps 6e-8 relative precision, far below the 1e-5 the
parity test asserts.  Runtime: about 13 minutes per value on 8 cores.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as wl                      # noqa: E402
from oracle import asn_oracle as o          # noqa: E402

OUT = os.path.join(HERE, "line_source_400_q512_phi.npz")
SIGMA_AS = (0.0, 1.0, 5.0)


def main():
    arrays = {}
    for s in SIGMA_AS:
        spec = wl.line_source(400, n_polar=16, sigma_as=s, beta=4.5)
        t0 = time.time()
        psi, st, _ = o.run(spec)
        phi = o.scalar_flux(psi, st.w)
        arrays[f"phi_as{int(s)}"] = phi.astype(np.float32)
        arrays["n_steps"] = np.array(st.n_steps)
        arrays["dt"] = np.array(st.dt)
        print(f"sigma_as {s}: {st.n_steps} steps, dt {st.dt:.9g}, mass {phi.sum() * st.dx * st.dy:.9g}, "
              f"{time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(OUT, **arrays)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
