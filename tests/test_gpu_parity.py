"""GPU parity against the FP64 oracle, through the C ABI.

Bars: streaming bit exact in every storage type; F64 collision, init,
moments and multi-step runs within 1e-12 (normwise relative, per Pauli
component); F32 storage within 1e-5 after the configured steps; F16 scaled
deviation compared population by population and on the cell density
matrices, against bounds set from the measured errors.  Sizes span several thread
blocks with ragged edges.
"""
import numpy as np
import pytest
import torch

from helpers import (decode_f16dev, device_inputs, f16dev_rounding_bound, fields, from_pauli, gpu_init, make_handle,
                     normwise_rel_err, oracle_init, oracle_pauli, to_pauli_np)
from oracle import pauli, qlbm
from paper_1309_1656_amd import mlbm

pytestmark = pytest.mark.gpu

SHAPES = [(64, 64), (37, 70), (1, 5), (13, 9, 11), (6, 5, 70), (1, 1, 1)]

# F16 scaled-deviation storage after tens to hundreds of steps, normwise against the FP64 oracle:
# populations and cell density matrices
F16_POP_BAR = 1e-2
F16_RHO_BAR = 5e-3


def _flush(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("storage", [mlbm.MLBM_STORE_F64, mlbm.MLBM_STORE_F32, mlbm.MLBM_STORE_F16DEV])
def test_stream_bit_exact(shape, storage):
    _flush(f"stream {shape} storage={storage}")
    h = make_handle(shape, storage=storage)
    rng = np.random.default_rng(3)
    host = rng.standard_normal(h.field_shape)
    src = torch.from_numpy(host).to(h.field_dtype).cuda()
    dst = h.empty_field()
    mlbm.mlbm_stream(h, src, dst)
    torch.cuda.synchronize()
    lat = qlbm.Lattice(len(shape))
    raw = h.pauli_view(src).cpu().numpy()
    expect = np.stack([qlbm.stream(lat, raw[k][..., None, None])[..., 0, 0] for k in range(4)])
    got = np.ascontiguousarray(h.pauli_view(dst).cpu().numpy())
    assert got.dtype == expect.dtype
    assert np.array_equal(got.view(np.uint8), expect.view(np.uint8))


@pytest.mark.parametrize("shape", [(37, 70), (13, 9, 11), (6, 5, 70)])
def test_init_matches_oracle(shape):
    _flush(f"init {shape}")
    f = fields(shape, 21)
    h = make_handle(shape)
    W = to_pauli_np(h, gpu_init(h, f))
    _, Wo = oracle_init(shape, f)
    assert normwise_rel_err(W, oracle_pauli(Wo)) < 1e-13


def test_init_degenerate_states_use_quadrature_branch():
    """nu > -1 exercises the trapezoidal Fermi-Dirac integrals (3D) and F_1 (2D)."""
    for shape in [(4, 5), (3, 4, 5)]:
        _flush(f"init degenerate {shape}")
        f = fields(shape, 5)
        f = dict(f)
        f["trrho"] = 6.0 + 2.0 * (f["trrho"] - 1.0) * 10
        f["r"] = f["r"] / np.abs(f["r"]).max() * 1.5
        f["T"] = 0.3 + 0.5 * (f["T"] - 1.0)
        h = make_handle(shape)
        W = to_pauli_np(h, gpu_init(h, f))
        lat, Wo = oracle_init(shape, f)
        _, nu_up, nu_dn, _ = qlbm.fd_parameters(lat.d, f["trrho"], f["r"], f["T"])
        assert nu_up.max() > 0.0     # degenerate regime reached
        assert normwise_rel_err(W, oracle_pauli(Wo)) < 1e-13


def _perturbed(lat, W, seed=5, amp=0.02):
    rng = np.random.default_rng(seed)
    a = rng.normal(0, amp, size=(4,) + W.shape[:-2]) * lat.w.reshape((1, -1) + (1,) * lat.d)
    return W + pauli.matrix_from_pauli(a)


@pytest.mark.parametrize("shape", [(37, 70), (13, 9, 11)])
@pytest.mark.parametrize("inplace", [False, True])
def test_collide_matches_oracle(shape, inplace):
    _flush(f"collide {shape} inplace={inplace}")
    f = fields(shape, 8)
    lat, Wo = oracle_init(shape, f)
    Wo = _perturbed(lat, Wo)
    h = make_handle(shape, tau=0.7)
    src = from_pauli(h, oracle_pauli(Wo))
    dst = src if inplace else h.empty_field()
    mlbm.mlbm_collide(h, src, dst)
    got = to_pauli_np(h, dst)
    assert normwise_rel_err(got, oracle_pauli(qlbm.collide(lat, Wo, 0.7))) < 1e-14


@pytest.mark.parametrize("shape,steps,tau", [((64, 64), 100, 0.8), ((37, 70), 61, 0.6),
                                              ((13, 9, 11), 40, 0.8), ((6, 5, 70), 25, 1.0),
                                              # one row / one plane: the y (and z) neighbours wrap onto the cell's own row
                                              ((1, 300), 30, 0.8), ((1, 1, 300), 20, 0.7), ((2, 1, 129), 20, 0.9)])
def test_multi_step_f64(shape, steps, tau):
    _flush(f"steps f64 {shape} n={steps}")
    f = fields(shape, 1)
    h = make_handle(shape, tau=tau)
    W = gpu_init(h, f)
    mlbm.mlbm_step(h, W, h.empty_field(), steps)
    lat, Wo = oracle_init(shape, f)
    ref = oracle_pauli(qlbm.run(lat, Wo, tau, steps))
    assert normwise_rel_err(to_pauli_np(h, W), ref) < 1e-12


@pytest.mark.parametrize("shape,steps", [((64, 64), 100), ((13, 9, 11), 40)])
def test_multi_step_f32(shape, steps):
    _flush(f"steps f32 {shape} n={steps}")
    f = fields(shape, 1)
    h = make_handle(shape, storage=mlbm.MLBM_STORE_F32)
    W = gpu_init(h, f)
    mlbm.mlbm_step(h, W, h.empty_field(), steps)
    lat, Wo = oracle_init(shape, f)
    err = normwise_rel_err(to_pauli_np(h, W), oracle_pauli(qlbm.run(lat, Wo, 0.8, steps)))
    _flush(f"  f32 max rel err {err:.3e}")
    assert err < 1e-5


@pytest.mark.parametrize("shape,steps", [((64, 64), 100), ((13, 9, 11), 40)])
def test_multi_step_f16dev(shape, steps):
    """F16 scaled-deviation storage against the FP64 oracle, population by population (every stored
    value decoded as a = R_ki + s_i h) and on the cell density matrices."""
    _flush(f"steps f16dev {shape} n={steps}")
    f = fields(shape, 1)
    h = make_handle(shape, storage=mlbm.MLBM_STORE_F16DEV)
    W = gpu_init(h, f)
    assert h.info["f16_scale"] > 0
    lat, Wo = oracle_init(shape, f)
    # the initial state: one encoding of the oracle's values, each within half a unit in the last place
    a0, ref0 = decode_f16dev(h, W), oracle_pauli(Wo)
    assert np.all(np.abs(a0 - ref0) <= f16dev_rounding_bound(h, ref0) + 4e-7 * np.abs(ref0).max())
    mlbm.mlbm_step(h, W, h.empty_field(), steps)
    rho4 = torch.empty((4,) + tuple(shape), dtype=torch.float64, device="cuda")
    mlbm.mlbm_moments(h, W, rho4=rho4)
    Wn = qlbm.run(lat, Wo, 0.8, steps)
    rho_o, _, _, _ = qlbm.moments(lat, Wn)
    ref = pauli.pauli_from_matrix(rho_o)
    err_rho = max(np.abs(rho4.cpu().numpy()[k] - ref[k]).max() / np.abs(ref[k]).max() for k in range(4))
    err_pop = normwise_rel_err(decode_f16dev(h, W), oracle_pauli(Wn))
    _flush(f"  f16dev max rel err: populations {err_pop:.3e}, rho {err_rho:.3e}")
    assert err_pop < F16_POP_BAR
    assert err_rho < F16_RHO_BAR


@pytest.mark.parametrize("shape", [(37, 70), (13, 9, 11)])
def test_moments_match_oracle(shape):
    _flush(f"moments {shape}")
    f = fields(shape, 2)
    lat, Wo = oracle_init(shape, f)
    Wo = _perturbed(lat, Wo, amp=0.3)
    h = make_handle(shape)
    W = from_pauli(h, oracle_pauli(Wo))
    d = len(shape)
    rho4 = torch.empty((4,) + tuple(shape), dtype=torch.float64, device="cuda")
    u = torch.empty((d,) + tuple(shape), dtype=torch.float64, device="cuda")
    eps = torch.empty(tuple(shape), dtype=torch.float64, device="cuda")
    g8, nneg = mlbm.mlbm_moments(h, W, rho4, u, eps)
    rho, T, uo, eo = qlbm.moments(lat, Wo)
    assert np.max(np.abs(rho4.cpu().numpy() - pauli.pauli_from_matrix(rho))) < 1e-14
    assert np.max(np.abs(u.cpu().numpy() - uo)) < 1e-14
    assert np.max(np.abs(eps.cpu().numpy() - eo)) < 1e-13
    go = qlbm.global_means(lat, Wo)
    assert np.max(np.abs(g8 - go)) < 1e-14 * np.abs(go).max()
    assert nneg == qlbm.count_negative_eigenvalues(Wo)
    assert nneg > 0      # the perturbation is large enough to produce some


def test_nonfinite_is_reported():
    shape = (16, 16)
    h = make_handle(shape)
    W = gpu_init(h, fields(shape, 3))
    W[3, 0, 5, 7] = float("nan")
    with pytest.raises(mlbm.MlbmError) as e:
        mlbm.mlbm_moments(h, W)
    assert e.value.code == mlbm.MLBM_ENONFINITE


@pytest.mark.parametrize("bad", ["T", "r", "trrho", "nan"])
def test_init_domain_errors(bad):
    shape = (8, 9)
    f = {k: v.copy() for k, v in fields(shape, 4).items()}
    if bad == "T":
        f["T"][2, 3] = -0.1
    elif bad == "r":
        f["r"][:, 4, 4] = [f["trrho"][4, 4], 0.0, 0.0]
    elif bad == "trrho":
        f["trrho"][0, 0] = 0.0
    else:
        f["u_lat"][0, 1, 1] = float("nan")
    h = make_handle(shape)
    with pytest.raises(mlbm.MlbmError) as e:
        gpu_init(h, f)
    assert e.value.code == mlbm.MLBM_EDOMAIN


def test_determinism_bitwise():
    shape = (13, 9, 11)
    f = fields(shape, 6)
    outs = []
    for _ in range(2):
        h = make_handle(shape)
        W = gpu_init(h, f)
        mlbm.mlbm_step(h, W, h.empty_field(), 17)
        g8, _ = mlbm.mlbm_moments(h, W)
        outs.append((W.cpu().numpy(), g8))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_eigen_mode_equals_direct_and_oracle():
    for shape, steps in [((12, 10), 5), ((5, 6, 7), 3)]:
        _flush(f"eigen {shape}")
        f = fields(shape, 9)
        h = make_handle(shape)
        W = gpu_init(h, f)
        We = W.clone()
        mlbm.mlbm_step(h, W, h.empty_field(), steps)
        mlbm.mlbm_set_eq_mode(h, mlbm.MLBM_EQ_EIGEN)
        mlbm.mlbm_step(h, We, h.empty_field(), steps)
        a, b = to_pauli_np(h, W), to_pauli_np(h, We)
        assert normwise_rel_err(b, a) < 1e-12
        # one eigen-mode collision against the oracle's eigen route
        from oracle import eigen
        lat, Wo = oracle_init(shape, f)
        Wo = _perturbed(lat, Wo)
        src = from_pauli(h, oracle_pauli(Wo))
        dst = h.empty_field()
        mlbm.mlbm_collide(h, src, dst)
        ref = Wo + (1.0 / 0.8) * (eigen.equilibrium_eigen(lat, Wo) - Wo)
        assert normwise_rel_err(to_pauli_np(h, dst), oracle_pauli(ref)) < 1e-12


def test_resume_is_bitwise():
    """n1 steps, copy out, new handle, n2 steps == n1 + n2 steps (F16 reference restored)."""
    shape = (13, 9, 11)
    f = fields(shape, 7)
    for storage in (mlbm.MLBM_STORE_F64, mlbm.MLBM_STORE_F16DEV):
        h = make_handle(shape, storage=storage)
        W = gpu_init(h, f)
        Wa = W.clone()
        mlbm.mlbm_step(h, Wa, h.empty_field(), 12)
        mlbm.mlbm_step(h, W, h.empty_field(), 5)
        saved = W.cpu()
        h2 = make_handle(shape, storage=storage)
        if storage == mlbm.MLBM_STORE_F16DEV:
            mlbm.mlbm_set_f16_reference(h2, h.info["f16_ref"], h.info["f16_scale"])
        Wb = saved.cuda()
        mlbm.mlbm_step(h2, Wb, h2.empty_field(), 7)
        assert torch.equal(Wa, Wb)


@pytest.mark.parametrize("shape", [(37, 70), (13, 9, 130), (5, 6, 1)])
@pytest.mark.parametrize("storage", [mlbm.MLBM_STORE_F64, mlbm.MLBM_STORE_F32, mlbm.MLBM_STORE_F16DEV])
def test_launch_shapes_give_identical_results(shape, storage):
    """Every block width, XCD order, occupancy cap and store policy computes the same
    field, bit for bit (the shapes only reorder independent cells); ragged rows included."""
    _flush(f"launch shapes {shape} storage={storage}")
    f = fields(shape, 19)
    h = make_handle(shape, storage=storage)
    W0 = gpu_init(h, f)
    ref = None
    for stores in (0, 1):
        mlbm.mlbm_set_store_policy(h, stores)
        assert h.info["launch_temporal_stores"] == stores
        for bx in (64, 128):
            for order in (mlbm.MLBM_ORDER_NATURAL, mlbm.MLBM_ORDER_XCD_RANGE, mlbm.MLBM_ORDER_INTERLEAVE8):
                for cap in (0, 2):
                    mlbm.mlbm_set_launch(h, bx, order, cap)
                    W = W0.clone()
                    mlbm.mlbm_step(h, W, h.empty_field(), 3)
                    torch.cuda.synchronize()
                    if ref is None:
                        ref = W
                    else:
                        assert torch.equal(W, ref), (stores, bx, order, cap)


@pytest.mark.parametrize("shape", [(37, 70), (13, 9, 130)])
@pytest.mark.parametrize("feature", ["field_map", "isothermal", "positivity"])
def test_launch_shapes_give_identical_results_with_features(shape, feature):
    """The magnetic-field and variant kernels under every launch shape: the
    variants always run 64-cell blocks, the field kernels both widths."""
    _flush(f"launch shapes {shape} {feature}")
    f = fields(shape, 23)
    h = make_handle(shape)
    if feature == "field_map":
        bmap = torch.from_numpy(np.random.default_rng(8).normal(0, 0.05, size=(3,) + tuple(shape))).cuda()
        mlbm.mlbm_set_magnetic_field_map(h, bmap)
    elif feature == "isothermal":
        mlbm.mlbm_set_eq_mode(h, mlbm.MLBM_EQ_ISOTHERMAL)
    else:
        mlbm.mlbm_set_positivity(h, 1)
    W0 = gpu_init(h, f)
    if feature == "positivity":
        # nearly pure spin states (|a_k| = 0.97 a_0 per population), so that the limit acts
        a = to_pauli_np(h, W0)
        dirs = np.random.default_rng(9).normal(size=(3,) + a.shape[1:])
        a[1:] = 0.97 * a[0][None] * dirs / np.linalg.norm(dirs, axis=0)
        W0 = from_pauli(h, a)
    ref = None
    for bx in (64, 128):
        for order in (mlbm.MLBM_ORDER_NATURAL, mlbm.MLBM_ORDER_XCD_RANGE, mlbm.MLBM_ORDER_INTERLEAVE8):
            for cap in (0, 2):
                mlbm.mlbm_set_launch(h, bx, order, cap)
                W = W0.clone()
                mlbm.mlbm_step(h, W, h.empty_field(), 3)
                torch.cuda.synchronize()
                if ref is None:
                    ref = W
                else:
                    assert torch.equal(W, ref), (bx, order, cap)
    if feature == "positivity":
        mlbm.mlbm_set_positivity(h, 0)
        W = W0.clone()
        mlbm.mlbm_step(h, W, h.empty_field(), 3)
        assert not torch.equal(W, ref)      # the limit acted


@pytest.mark.parametrize("nbytes", [16, 4096 + 16, (1 << 20) + 48])
def test_device_copy_is_exact(nbytes):
    """The diagnostic copy moves exactly nbytes and touches nothing after them."""
    _flush(f"device copy {nbytes} bytes")
    gen = torch.Generator(device="cuda").manual_seed(nbytes)
    src = torch.randint(0, 256, (nbytes + 64,), dtype=torch.uint8, device="cuda", generator=gen)
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
    mlbm.mlbm_device_copy(src, dst, nbytes)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src[:nbytes])
    assert int(dst[nbytes:].count_nonzero()) == 0


@pytest.mark.parametrize("shape", [(37, 70), (13, 9, 130), (3, 5, 100)])
@pytest.mark.parametrize("storage", [mlbm.MLBM_STORE_F64, mlbm.MLBM_STORE_F32, mlbm.MLBM_STORE_F16DEV])
@pytest.mark.parametrize("feature", [None, "field_map", "field_uniform", "isothermal", "positivity", "iso_pos", "eigen"])
def test_step_equals_single_steps(shape, storage, feature):
    """mlbm_step(n) for n >= 2 ends with a pass that collides and pushes straight into W; mlbm_step(1) is the
    collide-only pass plus the stream-only pass.  n single steps give mlbm_step(n) bit for bit (n odd and even,
    so the collide-only pass runs both in place and out of place), with every collision kind."""
    if feature == "eigen" and storage != mlbm.MLBM_STORE_F64:
        pytest.skip("the eigen-channel mode runs on F64 storage only")
    _flush(f"step(n) == n x step(1) {shape} storage={storage} feature={feature}")
    f = fields(shape, 29)
    h = make_handle(shape, storage=storage)
    if feature == "field_map":
        bmap = torch.from_numpy(np.random.default_rng(3).normal(0, 0.05, size=(3,) + tuple(shape))).cuda()
        mlbm.mlbm_set_magnetic_field_map(h, bmap)
    elif feature == "field_uniform":
        mlbm.mlbm_set_magnetic_field(h, [0.02, -0.03, 0.01])
    elif feature in ("isothermal", "iso_pos"):
        mlbm.mlbm_set_eq_mode(h, mlbm.MLBM_EQ_ISOTHERMAL)
    elif feature == "eigen":
        mlbm.mlbm_set_eq_mode(h, mlbm.MLBM_EQ_EIGEN)
    if feature in ("positivity", "iso_pos"):
        mlbm.mlbm_set_positivity(h, 1)
    W0 = gpu_init(h, f)
    scratch = h.empty_field()
    for n in (2, 3, 5, 6):
        A = W0.clone()
        mlbm.mlbm_step(h, A, scratch, n)
        B = W0.clone()
        for _ in range(n):
            mlbm.mlbm_step(h, B, scratch, 1)
        torch.cuda.synchronize()
        assert torch.equal(A, B), n
