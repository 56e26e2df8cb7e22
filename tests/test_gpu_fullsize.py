"""Full-size workloads in the launch configuration the benchmark times.

For each workload:
* global conserved averages (Eqs. GlobalDensity, GlobalVelocity,
  GlobalTotalEnergy) stay constant over the whole run;
* the last step is checked cell by cell at sampled cells against one oracle
  step computed from the GPU's own state before it (the oracle collides the
  Q neighbour cells x - c_i and streams population i to x); F16
  scaled-deviation values are decoded first and held to their encoding
  rounding;
* where a stored oracle run exists (tests/golden/oracle_<name>.npz, written
  by tests/golden/make_oracle_runs.py), the final state is compared with it at
  the stored cells: F64 within 1e-12, F32 within 1e-5, F16 scaled deviation
  population by population within F16_POP_BAR (normwise: max error over the
  sampled populations / max |a_k| over the whole field).
"""
import os

import numpy as np
import pytest
import torch

from helpers import dims_of, f16dev_rounding_bound, f16dev_scales, make_handle
from oracle import pauli, qlbm
from paper_1309_1656_amd import mlbm, synthetic

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
B = synthetic.BASE_SEED

# F16 scaled-deviation storage against the FP64 oracle after the configured steps (normwise, per
# Pauli component): populations, cell density matrices, and the relative drift of the global averages
F16_POP_BAR = 1e-2
F16_RHO_BAR = 5e-3
F16_DRIFT_BAR = 1e-4


def _log(msg):
    print(msg, flush=True)


def _inputs(h, f):
    to = lambda a: (a if torch.is_tensor(a) else torch.from_numpy(np.ascontiguousarray(a))).to(
        device="cuda", dtype=torch.float64).contiguous()
    rho4 = torch.cat([to(f["trrho"])[None], to(f["r"])])
    return rho4, to(f["u_lat"]) * h.info["xi"], to(f["T"])


def _cells(shape, flat):
    return np.unravel_index(flat, shape)


def _gather(h, W, idx):
    """Values [4, Q, M] of field W at the cells idx (tuple of index arrays per grid axis), decoded
    for F16 scaled-deviation storage."""
    sel = h.pauli_view(W)[(slice(None), slice(None)) + tuple(torch.from_numpy(np.asarray(c)).cuda() for c in idx)]
    if h.info["storage"] != mlbm.MLBM_STORE_F16DEV:
        return sel.to(torch.float64).cpu().numpy()
    Q = h.Q
    hv = sel.cpu().numpy().astype(np.float32)
    ref = np.asarray(h.info["f16_ref"], dtype=np.float32).reshape(4, Q, 1)
    sc = f16dev_scales(h).astype(np.float32).reshape(1, Q, 1)
    return (ref + sc * hv).astype(np.float64)


def sampled_step_check(h, W_before, W_after, tau, ncheck=512, seed=0):
    """One GPU step at sampled cells against the oracle: the oracle collides every sampled cell x of
    the GPU's state before the step, and population i of the result must be found at x + c_i after
    it (the streaming of Eq. TransportStep).

    Returns (normwise error, worst ratio of |error| to the per-value allowance).  The ratio is 0 for
    F64 and F32, which only use the normwise error.  For F16 scaled-deviation storage the allowance
    is the encoding rounding of the value (half a unit in the last place of its half-precision
    deviation, times s_i; the larger of those at the expected and at the stored value) plus 1e-6 of
    the component's scale for the float arithmetic of the collision."""
    shape = h.grid
    d = len(shape)
    lat = qlbm.Lattice(d, h.info["beta0"])
    Q = lat.Q
    rng = np.random.default_rng(seed)
    flat = rng.choice(int(np.prod(shape)), ncheck, replace=False)
    coords = _cells(shape, flat)
    a = _gather(h, W_before, coords)                                                 # [4, Q, M]
    expect = pauli.pauli_from_matrix(qlbm.collide(lat, pauli.matrix_from_pauli(a), tau))
    # population i of x's collision sits at x + c_i after the step (array axis ax <-> component d-1-ax)
    nb = [((coords[ax][:, None] + lat.c[None, :, d - 1 - ax]) % shape[ax]).reshape(-1) for ax in range(d)]
    got_all = _gather(h, W_after, nb).reshape(4, Q, ncheck, Q)
    got = np.diagonal(got_all, axis1=1, axis2=3).transpose(0, 2, 1)                 # [4, Q, M]
    scale = np.abs(expect).reshape(4, -1).max(axis=1)
    err = max(np.abs(got[k] - expect[k]).max() / scale[k] for k in range(4))
    ratio = 0.0
    if h.info["storage"] == mlbm.MLBM_STORE_F16DEV:
        rb = np.maximum(f16dev_rounding_bound(h, expect), f16dev_rounding_bound(h, got))
        ratio = float((np.abs(got - expect) / (rb + 1e-6 * scale.reshape(4, 1, 1))).max())
    return err, ratio


def sampled_step_error(h, W_before, W_after, tau, ncheck=512, seed=0):
    """Normwise error of one GPU step at sampled cells against the oracle (F64, F32)."""
    return sampled_step_check(h, W_before, W_after, tau, ncheck, seed)[0]


def golden_error(h, W, name):
    path = os.path.join(GOLDEN, f"oracle_{name}.npz")
    if not os.path.exists(path):
        return None
    g = np.load(path)
    coords = _cells(h.grid, g["cells"])
    idx = tuple(torch.from_numpy(c).cuda() for c in coords)
    got = h.pauli_view(W)[(slice(None), slice(None)) + idx].to(torch.float64).cpu().numpy()
    ref = g["values"]
    return max(np.abs(got[k] - ref[k]).max() / g["maxabs"][k] for k in range(4))


def golden_pop_error_f16(h, W, name):
    """F16 scaled-deviation storage: the decoded populations at the stored cells."""
    path = os.path.join(GOLDEN, f"oracle_{name}.npz")
    if not os.path.exists(path):
        return None
    g = np.load(path)
    got = _gather(h, W, _cells(h.grid, g["cells"]))
    ref = g["values"]
    return max(np.abs(got[k] - ref[k]).max() / g["maxabs"][k] for k in range(4))


def golden_rho_error(h, W, name):
    """F16 deviation storage: compare the density matrices at the stored cells."""
    path = os.path.join(GOLDEN, f"oracle_{name}.npz")
    if not os.path.exists(path):
        return None
    g = np.load(path)
    rho4 = torch.empty((4,) + tuple(h.grid), dtype=torch.float64, device="cuda")
    mlbm.mlbm_moments(h, W, rho4=rho4)
    coords = _cells(h.grid, g["cells"])
    idx = tuple(torch.from_numpy(c).cuda() for c in coords)
    got = rho4[(slice(None),) + idx].cpu().numpy()
    ref = g["values"].sum(axis=1)
    return max(np.abs(got[k] - ref[k]).max() / np.abs(ref[k]).max() for k in range(4))


def run_workload(shape, tau, steps, f, storage, name=None, sampled=True):
    h = make_handle(shape, tau=tau, storage=storage)
    W = h.empty_field()
    mlbm.mlbm_init_equilibrium(h, W, *_inputs(h, f))
    g0, _ = mlbm.mlbm_moments(h, W)
    scratch = h.empty_field()
    mlbm.mlbm_step(h, W, scratch, steps - 1)
    Wb = W.clone() if sampled else None
    mlbm.mlbm_step(h, W, scratch, 1)
    g1, nneg = mlbm.mlbm_moments(h, W)
    out = {"drift": float(np.abs(g1 - g0).max() / np.abs(g0).max()), "n_neg": nneg}
    if sampled:
        out["step"], out["step_allowance_ratio"] = sampled_step_check(h, Wb, W, tau)
    del Wb
    if name is not None:
        if storage != mlbm.MLBM_STORE_F16DEV:
            out["golden"] = golden_error(h, W, name)
        else:
            out["golden"] = golden_pop_error_f16(h, W, name)
            out["golden_rho"] = golden_rho_error(h, W, name)
    _log(f"{name or shape} storage={storage}: {out}")
    return h, W, out


@pytest.mark.parametrize("storage", [mlbm.MLBM_STORE_F64, mlbm.MLBM_STORE_F32, mlbm.MLBM_STORE_F16DEV])
def test_d3q19_128(storage):
    """D3Q19 128^3, tau 0.8, 500 steps: the benchmark workload."""
    shape = (128, 128, 128)
    f = synthetic.macroscopic_fields(shape, B + 3)
    _, _, r = run_workload(shape, 0.8, 500, f, storage, "d3q19_128_tau0.8_500")
    if storage == mlbm.MLBM_STORE_F64:
        assert r["drift"] < 1e-12 and r["step"] < 1e-13
        assert r["golden"] is None or r["golden"] < 1e-12
    elif storage == mlbm.MLBM_STORE_F32:
        assert r["drift"] < 1e-8 and r["step"] < 1e-6
        assert r["golden"] is None or r["golden"] < 1e-5
    else:
        # one step: every value within its encoding rounding; 500 steps: populations and rho
        assert r["step_allowance_ratio"] <= 1.0
        assert r["drift"] < F16_DRIFT_BAR
        assert r["golden"] is None or r["golden"] < F16_POP_BAR
        assert r["golden_rho"] is None or r["golden_rho"] < F16_RHO_BAR


@pytest.mark.parametrize("storage", [mlbm.MLBM_STORE_F64, mlbm.MLBM_STORE_F32, mlbm.MLBM_STORE_F16DEV])
def test_d3q19_64_subrun(storage):
    """The 64^3 sub-run of the 384^3 workload family, 200 steps, against the stored oracle run."""
    shape = (64, 64, 64)
    f = synthetic.macroscopic_fields(shape, B + 4)
    _, _, r = run_workload(shape, 0.8, 200, f, storage, "d3q19_64_tau0.8_200")
    assert r["golden"] is not None, "stored oracle run missing"
    bar = {mlbm.MLBM_STORE_F64: 1e-12, mlbm.MLBM_STORE_F32: 1e-5, mlbm.MLBM_STORE_F16DEV: F16_POP_BAR}[storage]
    assert r["golden"] < bar
    if storage == mlbm.MLBM_STORE_F16DEV:
        assert r["golden_rho"] < F16_RHO_BAR and r["step_allowance_ratio"] <= 1.0


@pytest.mark.parametrize("storage", [mlbm.MLBM_STORE_F64, mlbm.MLBM_STORE_F32, mlbm.MLBM_STORE_F16DEV])
def test_d3q19_384(storage):
    """D3Q19 384^3, 200 steps: conservation and a sampled oracle step at full size."""
    shape = (384, 384, 384)
    f = synthetic.macroscopic_fields(shape, B + 4, device="cuda")
    h, W, r = run_workload(shape, 0.8, 200, f, storage, None)
    del f
    if storage == mlbm.MLBM_STORE_F64:
        assert r["drift"] < 1e-12 and r["step"] < 1e-13
    elif storage == mlbm.MLBM_STORE_F32:
        assert r["drift"] < 1e-8 and r["step"] < 1e-6
    else:
        assert r["drift"] < F16_DRIFT_BAR and r["step_allowance_ratio"] <= 1.0
    del W, h
    torch.cuda.empty_cache()


@pytest.mark.parametrize("storage", [mlbm.MLBM_STORE_F64, mlbm.MLBM_STORE_F32, mlbm.MLBM_STORE_F16DEV])
def test_d3q19_512_large(storage):
    """D3Q19 512^3 (134M cells; FP64: two 81.6 GB fields), 3 steps: the largest grid
    here, past 2^32 field elements.  Conservation, and a sampled oracle step in FP32
    (FP64 keeps no third field for it; FP16 deviation has no sampled check)."""
    shape = (512, 512, 512)
    f = synthetic.macroscopic_fields(shape, B + 6, device="cuda")
    sampled = storage == mlbm.MLBM_STORE_F32
    h = make_handle(shape, tau=0.8, storage=storage)
    W = h.empty_field()
    mlbm.mlbm_init_equilibrium(h, W, *_inputs(h, f))
    del f
    torch.cuda.empty_cache()
    g0, _ = mlbm.mlbm_moments(h, W)
    scratch = h.empty_field()
    mlbm.mlbm_step(h, W, scratch, 2)
    Wb = W.clone() if sampled else None
    mlbm.mlbm_step(h, W, scratch, 1)
    g1, nneg = mlbm.mlbm_moments(h, W)
    drift = float(np.abs(g1 - g0).max() / np.abs(g0).max())
    out = {"drift": drift, "n_neg": nneg}
    if sampled:
        out["step"] = sampled_step_error(h, Wb, W, 0.8)
    _log(f"(512, 512, 512) storage={storage}: {out}")
    assert nneg == 0
    if storage == mlbm.MLBM_STORE_F64:
        assert drift < 1e-13
    elif storage == mlbm.MLBM_STORE_F32:
        assert drift < 1e-9 and out["step"] < 1e-6
    else:
        assert drift < 1e-5          # half-precision quantisation of the deviations
    del W, scratch, Wb, h
    torch.cuda.empty_cache()


@pytest.mark.parametrize("tau", [0.6, 1.0])
@pytest.mark.parametrize("storage", [mlbm.MLBM_STORE_F64, mlbm.MLBM_STORE_F32])
def test_d2q9_1024_shear(tau, storage):
    """D2Q9 1024^2 with the spin-polarised shear band, 1000 steps."""
    shape = (1024, 1024)
    f = synthetic.shear_band_fields(shape, B + 2)
    _, _, r = run_workload(shape, tau, 1000, f, storage, f"d2q9_1024_shear_tau{tau}_1000")
    if storage == mlbm.MLBM_STORE_F64:
        assert r["drift"] < 1e-12 and r["step"] < 1e-13
        assert r["golden"] is None or r["golden"] < 1e-12
    else:
        assert r["drift"] < 1e-8 and r["step"] < 1e-6
        assert r["golden"] is None or r["golden"] < 1e-5


def test_d2q9_512_rollout_f32_vs_f64():
    """Differentiation workload: FP32 rollout (checkpoints every 20) against the FP64 one on the GPU."""
    from paper_1309_1656_amd.rollout import MLBMRollout
    wl = synthetic.WORKLOADS["d2q9_512_adjoint"]
    shape, tau, steps = wl["shape"], wl["tau"], wl["steps"]
    f = synthetic.macroscopic_fields(shape, wl["seed"])
    rt = torch.from_numpy(synthetic.target_bloch_field(shape, wl["seed"] + 100)).cuda()
    res = {}
    for storage in (mlbm.MLBM_STORE_F64, mlbm.MLBM_STORE_F32):
        h = make_handle(shape, tau=tau, storage=storage)
        W0 = h.empty_field()
        mlbm.mlbm_init_equilibrium(h, W0, *_inputs(h, f))
        W0.requires_grad_(True)
        tau_t = torch.tensor(tau, dtype=torch.float64, requires_grad=True)
        loss = MLBMRollout.apply(W0, tau_t, h, steps, 20, rt)
        loss.backward()
        res[storage] = (loss.item(), h.pauli_view(W0.grad).double().cpu().numpy(), tau_t.grad.item())
    l64, g64, t64 = res[mlbm.MLBM_STORE_F64]
    l32, g32, t32 = res[mlbm.MLBM_STORE_F32]
    gerr = max(np.abs(g32[k] - g64[k]).max() / np.abs(g64[k]).max() for k in range(4))
    _log(f"512^2 rollout: loss {l64:.6e} rel diff {abs(l32 / l64 - 1):.2e}; grad W0 {gerr:.2e}; "
         f"grad tau {t64:.6e} rel diff {abs(t32 / t64 - 1):.2e}")
    assert np.isfinite(g32).all() and abs(l32 / l64 - 1) < 1e-5 and gerr < 1e-4 and abs(t32 / t64 - 1) < 1e-4


def _rotation(seed):
    """A fixed proper rotation of the Bloch vectors (the SO(3) image of one SU(2) matrix)."""
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    return q if np.linalg.det(q) > 0 else -q


def _rotate_bloch(h, W, R):
    """Turn the Bloch part (a1, a2, a3) of every population by R, in place, in double."""
    v = h.pauli_view(W)
    a = v[1:4].to(torch.float64)
    Rt = torch.from_numpy(R).cuda()
    v[1:4] = torch.tensordot(Rt, a, dims=([1], [0])).to(v.dtype)


@pytest.mark.parametrize("storage", [mlbm.MLBM_STORE_F64, mlbm.MLBM_STORE_F32])
def test_d3q19_128_su2_covariance(storage):
    """At the benchmark's size and launch shape: rotating every Bloch vector by one R before
    50 steps equals rotating the result (conjugation by one SU(2) matrix commutes with the
    step).  FP64 within 1e-13 of the field scale, FP32 within 1e-6."""
    shape = (128, 128, 128)
    f = synthetic.macroscopic_fields(shape, B + 3)
    h = make_handle(shape, tau=0.8, storage=storage)
    W = h.empty_field()
    mlbm.mlbm_init_equilibrium(h, W, *_inputs(h, f))
    R = _rotation(5)
    Wr = W.clone()
    _rotate_bloch(h, Wr, R)
    scratch = h.empty_field()
    mlbm.mlbm_step(h, W, scratch, 50)
    mlbm.mlbm_step(h, Wr, scratch, 50)
    _rotate_bloch(h, W, R)
    a, b = h.pauli_view(W).to(torch.float64), h.pauli_view(Wr).to(torch.float64)
    err = max(float((a[k] - b[k]).abs().max() / a[k].abs().max()) for k in range(4))
    _log(f"128^3 covariance storage={storage}: {err:.3e}")
    assert err < (1e-13 if storage == mlbm.MLBM_STORE_F64 else 1e-6)


@pytest.mark.parametrize("storage", [mlbm.MLBM_STORE_F64, mlbm.MLBM_STORE_F32])
def test_d3q19_128_scalar_state_stays_scalar(storage):
    """Unpolarised cells (|s| = 0 everywhere): every Bloch coefficient stays exactly zero over
    100 steps at the benchmark's size (W proportional to the identity is closed under the step)."""
    shape = (128, 128, 128)
    f = synthetic.macroscopic_fields(shape, B + 3)
    f = dict(f, r=np.zeros_like(f["r"]))
    h = make_handle(shape, tau=0.8, storage=storage)
    W = h.empty_field()
    mlbm.mlbm_init_equilibrium(h, W, *_inputs(h, f))
    mlbm.mlbm_step(h, W, h.empty_field(), 100)
    v = h.pauli_view(W)
    assert int(v[1:4].count_nonzero()) == 0
    assert bool(torch.isfinite(v[0]).all())
