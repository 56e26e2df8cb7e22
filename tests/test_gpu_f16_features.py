"""FP16 scaled-deviation storage together with the features added to the
plain step: magnetic field, isothermal model, positivity limit and the
chemical-potential initial state.  Every stored value is decoded
(a = R_ki + s_i h) and compared with the oracle population by population, and
the cell density matrices rho = sum_i W_i are compared too (normwise, with
the bars of the plain FP16 runs).  The initial states are held to the
encoding rounding of each value.
"""
import numpy as np
import pytest
import torch

from helpers import decode_f16dev, f16dev_rounding_bound, fields, gpu_init, make_handle, normwise_rel_err, oracle_init
from oracle import magnetic, pauli, qlbm, variants
from paper_1309_1656_amd import mlbm

pytestmark = pytest.mark.gpu

F16 = mlbm.MLBM_STORE_F16DEV
F16_POP_BAR = 1e-2
F16_RHO_BAR = 5e-3


def _pop_err(h, W, ref_W):
    """Normwise error of the decoded populations."""
    return normwise_rel_err(decode_f16dev(h, W), pauli.pauli_from_matrix(ref_W))


def _rho_err(h, W, ref_W):
    """Normwise error of the decoded cell density matrices (mlbm_moments decodes the stored deviations)."""
    grid = h.grid
    rho4 = torch.empty((4,) + tuple(grid), dtype=torch.float64, device="cuda")
    mlbm.mlbm_moments(h, W, rho4=rho4)
    ref = pauli.pauli_from_matrix(ref_W.sum(axis=0))
    got = rho4.cpu().numpy()
    return np.abs(got - ref).max() / np.abs(ref).max()


@pytest.mark.parametrize("shape", [(37, 70), (13, 9, 11)])
@pytest.mark.parametrize("feature", ["field", "isothermal", "positivity"])
def test_f16_with_feature(shape, feature):
    print(f"f16 {feature} {shape}", flush=True)
    f = fields(shape, 23)
    lat, Wo = oracle_init(shape, f)
    tau, n = 0.8, 5
    h = make_handle(shape, tau=tau, storage=F16)
    W = gpu_init(h, f)                       # fixes the F16 reference and scale
    mu_b = np.random.default_rng(2).normal(0, 0.3, size=(3,) + shape)
    keep = None
    if feature == "field":
        keep = torch.from_numpy(mu_b).cuda()
        mlbm.mlbm_set_magnetic_field_map(h, keep)
        ref = magnetic.run_with_field(lat, Wo, tau, mu_b, n)
    elif feature == "isothermal":
        mlbm.mlbm_set_eq_mode(h, mlbm.MLBM_EQ_ISOTHERMAL)
        ref = variants.run_variant(lat, Wo, tau, n, isothermal=True)
    else:
        mlbm.mlbm_set_positivity(h, 1)
        ref = variants.run_variant(lat, Wo, tau, n, positive=True)
    mlbm.mlbm_step(h, W, h.empty_field(), n)
    torch.cuda.synchronize()
    err = _rho_err(h, W, ref)
    perr = _pop_err(h, W, ref)
    print(f"  population err {perr:.3e}, rho err {err:.3e}", flush=True)
    assert perr < F16_POP_BAR
    assert err < F16_RHO_BAR


def test_f16_init_chemical():
    shape = (13, 9, 11)
    rng = np.random.default_rng(4)
    nu = rng.uniform(-4.0, -1.0, size=(2,) + shape)
    T = rng.uniform(0.8, 1.2, size=shape)
    u_lat = rng.uniform(-0.05, 0.05, size=(3,) + shape)
    h = make_handle(shape, storage=F16)
    W = h.empty_field()
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    mlbm.mlbm_init_chemical(h, W, to(nu), to(h.info["xi"] * u_lat), to(T))
    torch.cuda.synchronize()
    lat = qlbm.Lattice(3)
    Wo = qlbm.init_chemical(lat, nu[0], nu[1], lat.xi * u_lat, T)
    assert h.info["f16_scale"] > 0
    err = _rho_err(h, W, Wo)
    perr = _pop_err(h, W, Wo)
    print(f"  population err {perr:.3e}, rho err {err:.3e}", flush=True)
    # one encoding of the equilibrium: every value within half a unit in the last place
    ref = pauli.pauli_from_matrix(Wo)
    assert np.all(np.abs(decode_f16dev(h, W) - ref) <= f16dev_rounding_bound(h, ref) + 4e-7 * np.abs(ref).max())
    assert err < F16_RHO_BAR
