"""Write sampled FP64 oracle results of the full-size workloads.

Runs the CPU oracle (nothing else) from the seeded synthetic initial state
for the configured number of steps and stores, in tests/golden/oracle_<name>.npz:
  cells     flat indices of 1024 sampled cells (seeded)
  values    Pauli coefficients [4, Q, 1024] of the final pre-collision state there
  maxabs    max |a_k| over the whole final field, per Pauli component k
  global0 / global1   the 8 global averages at the start and at the end
  meta      [tau, steps, beta0]
  relax_t / relax   (runs with `record`) qlbm.relaxation every `record` steps
The differentiation workload (ROLLOUTS) stores instead, in
tests/golden/oracle_<name>.npz:
  cells     flat indices of 1024 sampled cells (seeded)
  grad      Pauli coefficients [4, Q, 1024] of dL/da of the initial state there
  maxabs    max |dL/da_k| over the whole initial field, per Pauli component k
  loss, dtau   the loss L = mean |r - r_target|^2 after the steps, and dL/dtau
  meta      [tau, steps, beta0, checkpoint interval]
Its reverse pass keeps a checkpoint every `ckpt` steps and recomputes the
states of one segment at a time from it (the oracle's own step, so the
recomputed states equal the first ones exactly); memory stays at one field
per checkpoint plus one segment.
Usage: python tests/golden/make_oracle_runs.py [name ...]   (default: all)
These runs take from minutes (64^3, the 512^2 rollout) to over an hour
(128^3) on one core.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import adjoint, pauli, qlbm  # noqa: E402
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
ROLLOUTS = {
    "d2q9_512_rollout_tau0.8_200": dict(workload="d2q9_512_adjoint", ckpt=20),
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


def run_rollout(name):
    """dL/dW0 and dL/dtau of the spin-density loss after the differentiation workload's steps, by the
    oracle's step, loss and one-step adjoint, with checkpoints every cfg['ckpt'] steps."""
    cfg = ROLLOUTS[name]
    wl = synthetic.WORKLOADS[cfg["workload"]]
    shape, tau, steps, K = wl["shape"], wl["tau"], wl["steps"], cfg["ckpt"]
    lat = qlbm.Lattice(len(shape), 1.0)
    f = synthetic.macroscopic_fields(shape, wl["seed"])
    r_target = synthetic.target_bloch_field(shape, wl["seed"] + 100)
    t0 = time.time()
    W = qlbm.init_equilibrium(lat, f["trrho"], f["r"], lat.xi * f["u_lat"], f["T"])
    ckpts = {}
    for n in range(steps):
        if n % K == 0:
            ckpts[n] = W
        W = qlbm.step(lat, W, tau)
    loss, Lam = adjoint.spin_loss(lat, W, r_target)
    del W
    print(f"{name}: forward done ({time.time() - t0:.0f} s), loss {loss:.16e}", flush=True)
    dom = 0.0
    for start in sorted(ckpts, reverse=True):
        n_seg = min(K, steps - start)
        states = [ckpts.pop(start)]
        for _ in range(n_seg - 1):
            states.append(qlbm.step(lat, states[-1], tau))
        for j in range(n_seg - 1, -1, -1):
            Lam, d = adjoint.step_vjp(lat, states[j], Lam, tau)
            dom += d
        del states
        print(f"{name}: reverse segment from step {start} done ({time.time() - t0:.0f} s)", flush=True)
    dtau = -dom / tau ** 2
    grad = pauli.pauli_from_matrix(Lam) / 2.0         # dL/da_k of the Pauli coefficients
    cells = sample_cells(shape)
    flat = grad.reshape(4, lat.Q, -1)
    np.savez(os.path.join(HERE, f"oracle_{name}.npz"), cells=cells, grad=flat[:, :, cells],
             maxabs=np.abs(flat).max(axis=(1, 2)), loss=np.array(loss), dtau=np.array(dtau),
             meta=np.array([tau, steps, 1.0, K]))
    print(f"{name}: done in {time.time() - t0:.0f} s, dL/dtau {dtau:.16e}", flush=True)


if __name__ == "__main__":
    for nm in (sys.argv[1:] or list(RUNS) + list(ROLLOUTS)):
        if nm in ROLLOUTS:
            run_rollout(nm)
        else:
            run(nm)
