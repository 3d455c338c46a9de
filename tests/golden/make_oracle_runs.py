"""Write the FP64 oracle's state after long runs of the reduced workloads, for the GPU
parity tests whose oracle side takes minutes (1000 D3Q19 steps).

Each case is run by the oracle alone (`oracle/`), from the seeded inputs of
`pfinputs`, and stored as tests/golden/oracle_runs/<case>.npz with:
  phi [N], P [N], J [D][N]   the read-out after `steps` steps (float32; the parity bars
                             are 1e-5 in phi and 1e-4 relative in J, far above float32
                             rounding of the stored values)
  mass0, mass1               sum(phi) at the start and after `steps` steps (float64)
  steps                      the step count
  cfg                        the workload dict as JSON
  source_sha1                hash of the oracle's sources: a test refuses a fixture
                             written by another oracle
  input_sha1                 hash of the seeded start (phi, u, P) the run began from

Run:  python tests/golden/make_oracle_runs.py [case ...]
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import pfinputs  # noqa: E402
from oracle import pflbm as O  # noqa: E402

OUT = os.path.join(HERE, "oracle_runs")
SOURCES = ("oracle/lattice.py", "oracle/pflbm.py")

# reduced forms of the D3Q19 workloads (rho_H/rho_L = 1000)
CASES = {
    "rising_bubble_24": (lambda: pfinputs.rising_bubble(n=24, R=5.0), 1000),
    "droplet_impact_36x28x30": (
        lambda: pfinputs.droplet_impact(nx=36, ny=28, nz=30, R=8.0, film=6.0), 1000),
    # the dam break (walls, open top) at a fifth of its size, gravity raised five-fold
    # so that the column collapses within the run
    "dam_break_48x6x40": (
        lambda: pfinputs.dam_break(nx=48, ny=6, nz=40, H=20.0, L=16.0, g=2e-5), 500),
}


def source_sha1():
    h = hashlib.sha1()
    for f in SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def input_sha1(cfg):
    h = hashlib.sha1()
    for a in pfinputs.fields(cfg):
        h.update(np.ascontiguousarray(a if a is not None else np.zeros(0, np.float32)).tobytes())
    return h.hexdigest()[:16]


def cfg_json(cfg):
    return json.dumps(cfg, sort_keys=True, default=lambda v: list(v))


def make(name):
    make_cfg, steps = CASES[name]
    cfg = make_cfg()
    phi, u, P = pfinputs.fields(cfg)
    prm = O.Params.from_dict(pfinputs.model_params(cfg))
    h, g = O.init(prm, phi.astype(np.float64), u.astype(np.float64), P.astype(np.float64))
    m0 = O.mass(h)
    h, g = O.run(prm, h, g, steps)
    ro = O.read(prm, h, g)
    D = 3 if cfg["lattice"] == 19 else 2
    os.makedirs(OUT, exist_ok=True)
    np.savez_compressed(os.path.join(OUT, name + ".npz"),
                        phi=ro["phi"].astype(np.float32), P=ro["P"].astype(np.float32),
                        J=ro["J"][:D].astype(np.float32), mass0=np.float64(m0),
                        mass1=np.float64(O.mass(h)), steps=np.int64(steps),
                        cfg=np.array(cfg_json(cfg)), source_sha1=np.array(source_sha1()),
                        input_sha1=np.array(input_sha1(cfg)))
    print(f"{name}: {steps} steps, mass {m0:.12g} -> {O.mass(h):.12g}", flush=True)


def load(name):
    """The stored run of `name` and the workload it was made for."""
    make_cfg, steps = CASES[name]
    with np.load(os.path.join(OUT, name + ".npz"), allow_pickle=False) as z:
        d = {k: z[k] for k in z.files}
    return make_cfg(), steps, d


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(CASES)):
        make(n)
