"""Expected values for the 16-bit storage forms on the static-droplet workload
(32^3 periodic box, G = 3.6, tau = 1, sphere R = 8, densities 1.0 / 0.03
mirrored, seeded noise 1e-4 with seed 1000), 10^4 steps.  Calls the oracle
only.

1. config3_oracle_1e4.npz: the FP64 oracle's fields after 10^4 steps
   (float32 is ample for errors of 16-bit storage): rho[2][32][32][32], the
   post-collision barycentric velocity u[3][32][32][32], the masses at step 0
   and 10^4 (float64).

2. config3_rounding_model.json: the error 16-bit storage with stochastic
   rounding causes, from the oracle itself: the oracle runs again with every
   stored population, at t = 0 and after every step, rounded stochastically
   to the format -- to the upper of its two representable neighbours with
   probability equal to its distance from the lower one over their spacing
   (FP16: 10 fraction bits, subnormal spacing 2^-24; BF16: 7 fraction bits)
   -- applied to the stored value d = f - w_i rho_ref, three independent
   seeds per form.  Per seed: the field errors against run 1 (per-field max
   and RMS, split by phase), the mass drift, the displacement of the
   droplet's liquid centre and the errors left after translating the fields
   back by it (16-bit storage keeps neither the total momentum nor the
   droplet's position exactly).

Usage: python tests/golden/make_config3_oracle.py  (about 20 minutes, 13
oracle runs in 8 parallel processes)
"""
import json
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import lbm  # noqa: E402
from tests import cases  # noqa: E402
from tests.golden.errors import aligned_errors, field_errors  # noqa: E402

STEPS = 10000
HERE = os.path.dirname(os.path.abspath(__file__))
from tests.golden.errors import CONFIG3_MODEL as MODEL  # noqa: E402
from tests.golden.errors import CONFIG3_ORACLE as OUT  # noqa: E402
FORMS = {"f16": 10, "bf16": 7}  # explicit fraction bits
REFS = (0.0, 1.0)
SEEDS = 3


def ulp(d, bits, fmt):
    """Spacing of the format's representable numbers at |d|."""
    _, e = np.frexp(np.abs(d))  # |d| = m 2^e, m in [0.5, 1)
    sp = np.ldexp(1.0, e - 1 - bits)
    if fmt == "f16":
        sp = np.maximum(sp, 2.0 ** -24)  # subnormal spacing
    return np.where(d == 0, 1.0, sp)


def round_stochastic(f, rho_ref, bits, fmt, rng):
    """Every stored deviation d = f - w_i rho_ref rounded stochastically to
    the format (away from zero with probability frac(|d| / ulp))."""
    wref = lbm.W[None, :, None, None, None] * np.asarray(rho_ref, float)[:, None, None, None, None]
    d = f - wref
    sp = ulp(d, bits, fmt)
    q = np.abs(d) / sp
    lo = np.floor(q)
    up = rng.uniform(0.0, 1.0, size=d.shape) < (q - lo)
    return wref + np.sign(d) * (lo + up) * sp


def run(job):
    fmt, ref, seed = job
    c = cases.sphere_case()
    r = lbm.Run(c["rho"], c["mat"], cases.oracle_params(c))
    rng = np.random.Generator(np.random.PCG64(31000 + 100 * seed + 10 * int(ref) + (fmt == "bf16")))
    m0 = r.masses()
    if fmt is not None:
        r.f = round_stochastic(r.f, (ref, ref), FORMS[fmt], fmt, rng)
    for _ in range(STEPS):
        r.step(1)
        if fmt is not None:
            r.f = round_stochastic(r.f, (ref, ref), FORMS[fmt], fmt, rng)
    rho, u = lbm.fields(r.f, r.material)
    return job, rho, u, m0, r.masses()


def main():
    jobs = [(None, 0.0, 0)] + [(f, r, sd) for f in FORMS for r in REFS for sd in range(SEEDS)]
    with Pool(8) as pool:
        res = pool.map(run, jobs)
    (_, rho_o, u_o, m0, m_o) = res[0]
    np.savez_compressed(OUT, rho=rho_o.astype(np.float32), u=u_o.astype(np.float32), mass0=m0, mass=m_o,
                        steps=STEPS)
    model = {"steps": STEPS, "seeds": SEEDS,
             "model": "stochastic rounding of every stored population at every step (oracle, FP64)", "forms": {}}
    for (fmt, ref, seed), rho, u, _, m in res[1:]:
        e = field_errors(rho, u, rho_o, u_o, m, m_o)
        e["aligned"] = aligned_errors(rho, u, rho_o, u_o)
        model["forms"].setdefault(f"{fmt}|rho_ref={ref:g}", []).append(e)
    with open(MODEL, "w") as fh:
        json.dump(model, fh, indent=1, sort_keys=True)
    print(OUT, MODEL)


if __name__ == "__main__":
    main()
