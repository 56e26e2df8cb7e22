"""Write sampled FP64 oracle results of the full-size workloads.

Runs the CPU oracle (nothing else) from the seeded synthetic initial state
for the configured number of steps and stores, in tests/golden/oracle_<name>.npz:
  cells     flat indices of 1024 sampled cells (seeded)
  values    Pauli coefficients [4, Q, 1024] of the final pre-collision state there
  maxabs    max |a_k| over the whole final field, per Pauli component k
  global0 / global1   the 8 global averages at the start and at the end
  meta      [tau, steps, beta0]
  relax_t / relax   (runs with `record`) qlbm.relaxation every `record` steps
Usage: python tests/golden/make_oracle_runs.py [name ...]   (default: all)
These runs take from minutes (64^3) to over an hour (128^3) on one core.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import pauli, qlbm  # noqa: E402
from paper_1309_1656_amd import synthetic  # noqa: E402

B = synthetic.BASE_SEED
RUNS = {
    "d3q19_128_tau0.8_500": dict(shape=(128, 128, 128), tau=0.8, steps=500, seed=B + 3, gen="generic"),
    "d3q19_64_tau0.8_200": dict(shape=(64, 64, 64), tau=0.8, steps=200, seed=B + 4, gen="generic"),
    "d2q9_1024_shear_tau0.6_1000": dict(shape=(1024, 1024), tau=0.6, steps=1000, seed=B + 2, gen="shear"),
    "d2q9_1024_shear_tau1.0_1000": dict(shape=(1024, 1024), tau=1.0, steps=1000, seed=B + 2, gen="shear"),
    "d3q19_convergence_32_tau10_300": dict(shape=(32, 32, 32), tau=10.0, steps=300, seed=None, gen="dichotomic",
                                           record=10),
}
NSAMPLE = 1024


def inputs(cfg):
    if cfg["gen"] == "shear":
        return synthetic.shear_band_fields(cfg["shape"], cfg["seed"])
    if cfg["gen"] == "dichotomic":
        return synthetic.dichotomic_fields(cfg["shape"])
    return synthetic.macroscopic_fields(cfg["shape"], cfg["seed"])


def sample_cells(shape):
    return np.sort(np.random.default_rng(0).choice(int(np.prod(shape)), NSAMPLE, replace=False))


def run(name):
    cfg = RUNS[name]
    shape = cfg["shape"]
    lat = qlbm.Lattice(len(shape), 1.0)
    f = inputs(cfg)
    W = qlbm.init_equilibrium(lat, f["trrho"], f["r"], lat.xi * f["u_lat"], f["T"])
    g0 = qlbm.global_means(lat, W)
    t0 = time.time()
    rec = cfg.get("record")
    relax_t, relax = [0], []
    if rec:
        relax.append(qlbm.relaxation(lat, W))
    for n in range(cfg["steps"]):
        W = qlbm.step(lat, W, cfg["tau"])
        if rec and (n + 1) % rec == 0:
            relax_t.append(n + 1)
            relax.append(qlbm.relaxation(lat, W))
        if (n + 1) % 50 == 0:
            print(f"{name}: step {n + 1}/{cfg['steps']} ({time.time() - t0:.0f} s)", flush=True)
    g1 = qlbm.global_means(lat, W)
    a = pauli.pauli_from_matrix(W)
    del W
    cells = sample_cells(shape)
    flat = a.reshape(4, lat.Q, -1)
    np.savez(os.path.join(HERE, f"oracle_{name}.npz"), cells=cells, values=flat[:, :, cells],
             maxabs=np.abs(flat).max(axis=(1, 2)), global0=g0, global1=g1,
             meta=np.array([cfg["tau"], cfg["steps"], 1.0]),
             **({"relax_t": np.array(relax_t), "relax": np.array(relax)} if rec else {}))
    print(f"{name}: done in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    for nm in (sys.argv[1:] or list(RUNS)):
        run(nm)
