"""The C ABI without a GPU: the library loads, exports every function that
include/mlbm.h declares, validates arguments on the host, and computes the
same constants as the oracle (mlbm_create touches no device memory)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import lattice as olat
from oracle import qlbm
from paper_1309_1656_amd import mlbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mlbm.h")

pytestmark = pytest.mark.skipif(not os.path.exists(mlbm.LIB_PATH), reason="libmlbm.so not built")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mlbm_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    lib = ctypes.CDLL(mlbm.LIB_PATH)
    declared = _declared()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(mlbm.EXPORTS)


@pytest.mark.parametrize("lattice,d,dims", [(9, 2, (16, 12, 1)), (19, 3, (8, 7, 6))])
@pytest.mark.parametrize("beta0", [0.8, 1.0, 1.2])
def test_constants_match_oracle(lattice, d, dims, beta0):
    h = mlbm.mlbm_create(lattice, dims, 0.8, beta0, mlbm.MLBM_STORE_F64)
    info = h.info
    lat = qlbm.Lattice(d, beta0)
    assert info["d"] == d and info["ncell"] == int(np.prod(dims))
    assert abs(info["xi"] / lat.xi - 1) < 1e-15
    assert np.max(np.abs(info["w"] / lat.w - 1)) < 1e-15
    assert np.array_equal(info["c"][:, :d], olat.velocities(d))
    for key in ("a1_0", "a1_b", "a2_0", "a2_b", "a3", "a4", "a5"):
        assert abs(info[key] / lat.coef[key] - 1) < 1e-15, key
    assert abs(info["omega"] - 1 / 0.8) < 1e-16
    h.destroy()


def test_field_bytes():
    for storage, size in [(0, 8), (1, 4), (2, 2)]:
        h = mlbm.mlbm_create(19, (5, 6, 7), 0.8, 1.0, storage)
        assert mlbm.mlbm_field_bytes(h) == 4 * 19 * 5 * 6 * 7 * size


@pytest.mark.parametrize("args,code", [
    ((10, (8, 8, 1), 0.8, 1.0, 0), mlbm.MLBM_EINVAL),     # bad lattice
    ((9, (8, 8, 2), 0.8, 1.0, 0), mlbm.MLBM_EINVAL),      # D2Q9 with nz != 1
    ((9, (0, 8, 1), 0.8, 1.0, 0), mlbm.MLBM_EINVAL),      # empty grid
    ((19, (8, 8, 8), 0.8, 1.0, 3), mlbm.MLBM_EINVAL),     # bad storage
    ((19, (1 << 16, 1 << 10, 1 << 6), 0.8, 1.0, 0), mlbm.MLBM_EINVAL),   # 2^32 cells
    ((19, (8, 70000, 8), 0.8, 1.0, 0), mlbm.MLBM_EINVAL),  # ny too large
    ((9, ((1 << 29) + 1, 1, 1), 0.8, 1.0, 1), mlbm.MLBM_EINVAL),   # a row beyond 32-bit byte offsets
    ((9, (8, 8, 1), 0.5, 1.0, 0), mlbm.MLBM_EDOMAIN),     # tau = 1/2
    ((9, (8, 8, 1), float("nan"), 1.0, 0), mlbm.MLBM_EDOMAIN),
    ((9, (8, 8, 1), 0.8, 0.0, 0), mlbm.MLBM_EDOMAIN),     # beta0 = 0
    ((9, (8, 8, 1), 0.8, float("inf"), 0), mlbm.MLBM_EDOMAIN),
])
def test_create_rejects(args, code):
    with pytest.raises(mlbm.MlbmError) as e:
        mlbm.mlbm_create(*args)
    assert e.value.code == code
    assert mlbm.mlbm_last_error()


def test_host_side_validation():
    h = mlbm.mlbm_create(9, (8, 8, 1), 0.8, 1.0, mlbm.MLBM_STORE_F32)
    lib = mlbm.load_library()
    with pytest.raises(mlbm.MlbmError) as e:
        mlbm.mlbm_set_tau(h, 0.3)
    assert e.value.code == mlbm.MLBM_EDOMAIN
    with pytest.raises(mlbm.MlbmError) as e:
        mlbm.mlbm_set_eq_mode(h, mlbm.MLBM_EQ_EIGEN)      # eigen mode needs F64
    assert e.value.code == mlbm.MLBM_EINVAL
    with pytest.raises(mlbm.MlbmError):
        mlbm.mlbm_set_eq_mode(h, 7)
    # null / aliasing pointers are rejected before any device work
    assert lib.mlbm_step(h.ptr, None, None, 3, None) == mlbm.MLBM_EINVAL
    buf = ctypes.c_void_p(4096)
    assert lib.mlbm_step(h.ptr, buf, buf, 3, None) == mlbm.MLBM_EINVAL
    assert lib.mlbm_step(h.ptr, buf, ctypes.c_void_p(8192), -1, None) == mlbm.MLBM_EINVAL
    assert lib.mlbm_step(h.ptr, buf, ctypes.c_void_p(8192), 0, None) == mlbm.MLBM_OK   # no-op
    assert lib.mlbm_stream(h.ptr, buf, buf, None) == mlbm.MLBM_EINVAL
    assert lib.mlbm_adjoint_step(h.ptr, buf, buf, buf, None, None) == mlbm.MLBM_EINVAL
    assert lib.mlbm_init_equilibrium(h.ptr, buf, None, buf, buf, None) == mlbm.MLBM_EINVAL
    assert lib.mlbm_set_f16_reference(h.ptr, None, 1.0) == mlbm.MLBM_EINVAL
    assert lib.mlbm_get_info(None, None) == mlbm.MLBM_EINVAL
    h16 = mlbm.mlbm_create(9, (8, 8, 1), 0.8, 1.0, mlbm.MLBM_STORE_F16DEV)
    assert lib.mlbm_spin_loss(h16.ptr, buf, buf, None, None, None) == mlbm.MLBM_EINVAL
    ref = np.arange(36, dtype=np.float64)
    mlbm.mlbm_set_f16_reference(h16, ref, 0.25)
    assert h16.info["f16_scale"] == 0.25
    assert np.array_equal(h16.info["f16_ref"].ravel(), ref)
    with pytest.raises(mlbm.MlbmError):
        mlbm.mlbm_set_f16_reference(h16, ref, -1.0)


def test_set_launch_validation_and_info():
    h = mlbm.mlbm_create(19, (128, 128, 128), 0.8, 1.0, mlbm.MLBM_STORE_F64)
    assert h.info["launch_block_x"] in (64, 128)
    assert h.info["launch_order"] in (0, 1, 2)
    mlbm.mlbm_set_launch(h, 128, mlbm.MLBM_ORDER_XCD_RANGE)
    assert h.info["launch_block_x"] == 128 and h.info["launch_order"] == mlbm.MLBM_ORDER_XCD_RANGE
    for bad in [(32, 0, 0), (256, 0, 0), (64, 3, 0), (64, -2, 0), (64, 0, -2), (64, 0, 33)]:
        with pytest.raises(mlbm.MlbmError) as e:
            mlbm.mlbm_set_launch(h, *bad)
        assert e.value.code == mlbm.MLBM_EINVAL
    mlbm.mlbm_set_launch(h, 64, mlbm.MLBM_ORDER_NATURAL, 3)
    assert h.info["launch_blocks_per_cu"] == 3
    mlbm.mlbm_set_launch(h, 0, mlbm.MLBM_ORDER_AUTO)
    assert h.info["launch_block_x"] in (64, 128)
    assert h.info["launch_blocks_per_cu"] == 2          # FP64 D3Q19 above 64^3
    # the field and variant kernels stream and take their own order and cap (measured at D3Q19
    # 128^3 FP64); the variants always in 64-cell blocks
    shape_of = lambda i: (i["launch_block_x"], i["launch_order"], i["launch_blocks_per_cu"], i["launch_temporal_stores"])
    I8, NAT = mlbm.MLBM_ORDER_INTERLEAVE8, mlbm.MLBM_ORDER_NATURAL
    mlbm.mlbm_set_magnetic_field(h, [0.1, 0.0, 0.0])
    assert shape_of(h.info) == (64, I8, 2, 0)
    mlbm.mlbm_set_magnetic_field(h, None)
    mlbm.mlbm_set_eq_mode(h, mlbm.MLBM_EQ_ISOTHERMAL)
    assert shape_of(h.info) == (64, I8, 3, 0)
    mlbm.mlbm_set_positivity(h, 1)
    assert shape_of(h.info) == (64, NAT, 0, 0)
    mlbm.mlbm_set_eq_mode(h, mlbm.MLBM_EQ_DIRECT)
    assert shape_of(h.info) == (64, NAT, 3, 0)
    mlbm.mlbm_set_launch(h, 128, mlbm.MLBM_ORDER_AUTO, 1)       # an explicit cap holds for them too
    assert shape_of(h.info) == (64, NAT, 1, 0)
    mlbm.mlbm_set_positivity(h, 0)
    assert h.info["launch_block_x"] == 128 and h.info["launch_blocks_per_cu"] == 1
    # elsewhere (FP32, smaller grids) they run uncapped in the plain kernels' order
    h32 = mlbm.mlbm_create(19, (128, 128, 128), 0.8, 1.0, mlbm.MLBM_STORE_F32)
    plain_order = h32.info["launch_order"]
    mlbm.mlbm_set_positivity(h32, 1)
    assert shape_of(h32.info) == (64, plain_order, 0, 0)
    h64 = mlbm.mlbm_create(19, (64, 64, 64), 0.8, 1.0, mlbm.MLBM_STORE_F64)
    mlbm.mlbm_set_magnetic_field(h64, [0.0, 0.0, 0.1])
    assert h64.info["launch_blocks_per_cu"] == 0 and h64.info["launch_temporal_stores"] == 0


def test_magnetic_field_validation():
    lib = mlbm.load_library()
    h = mlbm.mlbm_create(19, (8, 7, 6), 0.8, 1.0, mlbm.MLBM_STORE_F64)
    mlbm.mlbm_set_magnetic_field(h, [0.1, 0.0, -0.2])
    # the field excludes the eigen-channel mode and the adjoint
    with pytest.raises(mlbm.MlbmError) as e:
        mlbm.mlbm_set_eq_mode(h, mlbm.MLBM_EQ_EIGEN)
    assert e.value.code == mlbm.MLBM_EINVAL
    buf = [ctypes.c_void_p(4096 * (j + 1)) for j in range(3)]
    # (the adjoint takes the field; only aliasing is checked here, which fails before any launch)
    assert lib.mlbm_adjoint_step(h.ptr, buf[0], buf[1], buf[1], None, None) == mlbm.MLBM_EINVAL
    with pytest.raises(mlbm.MlbmError):
        mlbm.mlbm_set_magnetic_field(h, [float("nan"), 0.0, 0.0])
    # switched off (None or zero): both are allowed again
    mlbm.mlbm_set_magnetic_field(h, [0.0, 0.0, 0.0])
    mlbm.mlbm_set_eq_mode(h, mlbm.MLBM_EQ_EIGEN)
    with pytest.raises(mlbm.MlbmError) as e:
        mlbm.mlbm_set_magnetic_field(h, [0.1, 0.2, 0.3])
    assert e.value.code == mlbm.MLBM_EINVAL
    assert lib.mlbm_set_magnetic_field_map(h.ptr, ctypes.c_void_p(4096)) == mlbm.MLBM_EINVAL
    mlbm.mlbm_set_eq_mode(h, mlbm.MLBM_EQ_DIRECT)
    assert lib.mlbm_set_magnetic_field_map(h.ptr, ctypes.c_void_p(4096)) == mlbm.MLBM_OK
    mlbm.mlbm_set_magnetic_field(h, None)
    assert lib.mlbm_set_magnetic_field(None, None) == mlbm.MLBM_EINVAL


def test_variant_validation():
    lib = mlbm.load_library()
    h = mlbm.mlbm_create(9, (8, 8, 1), 0.8, 1.0, mlbm.MLBM_STORE_F64)
    mlbm.mlbm_set_eq_mode(h, mlbm.MLBM_EQ_ISOTHERMAL)
    assert h.info["eq_mode"] == mlbm.MLBM_EQ_ISOTHERMAL
    with pytest.raises(mlbm.MlbmError):
        mlbm.mlbm_set_magnetic_field(h, [0.1, 0.0, 0.0])
    buf = [ctypes.c_void_p(4096 * (j + 1)) for j in range(3)]
    assert lib.mlbm_adjoint_step(h.ptr, buf[0], buf[1], buf[2], None, None) == mlbm.MLBM_EINVAL
    mlbm.mlbm_set_positivity(h, 1)
    with pytest.raises(mlbm.MlbmError):
        mlbm.mlbm_set_eq_mode(h, mlbm.MLBM_EQ_EIGEN)
    mlbm.mlbm_set_eq_mode(h, mlbm.MLBM_EQ_DIRECT)
    assert lib.mlbm_adjoint_step(h.ptr, buf[0], buf[1], buf[2], None, None) == mlbm.MLBM_EINVAL
    with pytest.raises(mlbm.MlbmError):
        mlbm.mlbm_set_positivity(h, 2)
    mlbm.mlbm_set_positivity(h, 0)
    mlbm.mlbm_set_magnetic_field(h, [0.1, 0.0, 0.0])
    with pytest.raises(mlbm.MlbmError):
        mlbm.mlbm_set_positivity(h, 1)
    with pytest.raises(mlbm.MlbmError):
        mlbm.mlbm_set_eq_mode(h, mlbm.MLBM_EQ_ISOTHERMAL)
    with pytest.raises(mlbm.MlbmError):
        mlbm.mlbm_set_eq_mode(h, 3)


def test_device_copy_validation():
    """Requirements of the diagnostic copy are checked on the host before anything is enqueued."""
    lib = mlbm.load_library()
    cases = [(0, 4096, 64, "null"), (4096, 0, 64, "null"), (4096, 8192, 24, "multiple of 16"),
             (4104, 8192, 64, "aligned"), (4096, 4160, 128, "overlap"), (4096, 1 << 40, (1 << 35) + 16, "2^35")]
    for src, dst, n, msg in cases:
        rc = lib.mlbm_device_copy(ctypes.c_void_p(src), ctypes.c_void_p(dst), n, None)
        assert rc == mlbm.MLBM_EINVAL, (src, dst, n)
        assert msg in mlbm.mlbm_last_error(), mlbm.mlbm_last_error()


def test_step_states_and_sweep_validation():
    """Argument checks of mlbm_step_states and mlbm_adjoint_sweep (nothing is enqueued)."""
    h = mlbm.mlbm_create(9, (8, 8, 1), 0.8, 1.0, mlbm.MLBM_STORE_F32)
    lib = mlbm.load_library()
    fb = 4 * 9 * 64 * 4
    src, dst = ctypes.c_void_p(1 << 20), ctypes.c_void_p(2 << 20)
    st = ctypes.c_void_p(4 << 20)
    cases = [
        ((h.ptr, None, dst, st, 2, 3, None), "null field"),
        ((h.ptr, src, src, st, 2, 3, None), "distinct"),
        ((h.ptr, src, dst, st, 2, -1, None), "nsteps"),
        ((h.ptr, src, dst, None, 2, 3, None), "null states"),
        ((h.ptr, src, dst, st, 1, 3, None), "nstates"),
        ((h.ptr, src, dst, st, 0, 1, None), "nstates"),
        ((h.ptr, ctypes.c_void_p((4 << 20) + fb), dst, st, 2, 3, None), "overlap"),
        ((h.ptr, src, ctypes.c_void_p((4 << 20) + fb // 2), st, 2, 3, None), "overlap"),
    ]
    for args, msg in cases:
        assert lib.mlbm_step_states(*args) == mlbm.MLBM_EINVAL, msg
        assert msg in mlbm.mlbm_last_error(), (msg, mlbm.mlbm_last_error())
    # a field just after the states does not overlap them (rejected only for the step count here)
    assert lib.mlbm_step_states(h.ptr, ctypes.c_void_p((4 << 20) + 2 * fb), dst, st, 2, -1, None) == mlbm.MLBM_EINVAL
    assert "nsteps" in mlbm.mlbm_last_error()
    lam, tmp = ctypes.c_void_p(8 << 20), ctypes.c_void_p(9 << 20)
    assert lib.mlbm_adjoint_sweep(h.ptr, src, None, 3, lam, tmp, None, None) == mlbm.MLBM_EINVAL
    assert lib.mlbm_adjoint_sweep(h.ptr, src, st, 3, lam, lam, None, None) == mlbm.MLBM_EINVAL
    assert lib.mlbm_adjoint_sweep(h.ptr, src, st, -2, lam, tmp, None, None) == mlbm.MLBM_EINVAL
    assert lib.mlbm_adjoint_sweep(h.ptr, src, None, 0, lam, tmp, None, None) == mlbm.MLBM_OK   # nothing to do
    h16 = mlbm.mlbm_create(9, (8, 8, 1), 0.8, 1.0, mlbm.MLBM_STORE_F16DEV)
    assert lib.mlbm_adjoint_sweep(h16.ptr, src, st, 3, lam, tmp, None, None) == mlbm.MLBM_EINVAL
    mlbm.mlbm_set_eq_mode(h, mlbm.MLBM_EQ_ISOTHERMAL)
    assert lib.mlbm_adjoint_sweep(h.ptr, src, st, 3, lam, tmp, None, None) == mlbm.MLBM_EINVAL
    assert "direct equilibrium" in mlbm.mlbm_last_error()


def test_store_policy():
    """Automatic store policy: temporal writes up to 192 MiB per field, streaming above; the
    field and variant kernels always stream; the setter validates its argument."""
    cases = [(19, (128, 128, 128), mlbm.MLBM_STORE_F64, 0), (19, (64, 64, 64), mlbm.MLBM_STORE_F64, 1),
             (9, (512, 512, 1), mlbm.MLBM_STORE_F32, 1), (9, (1024, 1024, 1), mlbm.MLBM_STORE_F64, 0),
             (9, (1024, 1024, 1), mlbm.MLBM_STORE_F32, 1), (19, (128, 128, 128), mlbm.MLBM_STORE_F16DEV, 0)]
    for Q, dims, st, want in cases:
        h = mlbm.mlbm_create(Q, dims, 0.8, 1.0, st)
        assert h.info["launch_temporal_stores"] == want, (Q, dims, st)
    h = mlbm.mlbm_create(19, (64, 64, 64), 0.8, 1.0, mlbm.MLBM_STORE_F64)
    mlbm.mlbm_set_store_policy(h, 0)
    assert h.info["launch_temporal_stores"] == 0
    mlbm.mlbm_set_store_policy(h, 1)
    assert h.info["launch_temporal_stores"] == 1
    mlbm.mlbm_set_magnetic_field(h, [0.0, 0.0, 0.1])
    assert h.info["launch_temporal_stores"] == 0
    for bad in (-2, 2):
        with pytest.raises(mlbm.MlbmError) as e:
            mlbm.mlbm_set_store_policy(h, bad)
        assert e.value.code == mlbm.MLBM_EINVAL


def test_adjoint_launch_shape():
    """Automatic adjoint shape: the channel form (D3Q19 8-row interleave, per-XCD row ranges from 2^24
    cells, FP64 64-cell blocks capped at 2 workgroups per CU, FP32 128-cell blocks; D2Q9 64-cell blocks,
    8-row interleave, per-XCD row ranges for FP64 below 2^20 cells) without a
    field, the cell form with one; the setter validates its arguments and mlbm_get_info reports the
    shape in effect."""
    h = mlbm.mlbm_create(19, (128, 128, 128), 0.8, 1.0, mlbm.MLBM_STORE_F64)
    i = h.info
    assert (i["adjoint_form"], i["adjoint_block_x"], i["adjoint_order"], i["adjoint_blocks_per_cu"]) == (
        mlbm.MLBM_ADJ_CHANNEL, 64, mlbm.MLBM_ORDER_INTERLEAVE8, 2)
    assert i["adjoint_temporal_stores"] == 0
    h19f32 = mlbm.mlbm_create(19, (128, 128, 128), 0.8, 1.0, mlbm.MLBM_STORE_F32)
    i = h19f32.info
    assert (i["adjoint_form"], i["adjoint_block_x"], i["adjoint_order"], i["adjoint_blocks_per_cu"]) == (
        mlbm.MLBM_ADJ_CHANNEL, 128, mlbm.MLBM_ORDER_INTERLEAVE8, 0)
    big = mlbm.mlbm_create(19, (384, 384, 384), 0.8, 1.0, mlbm.MLBM_STORE_F64)      # from 2^24 cells: per-XCD rows
    assert (big.info["adjoint_block_x"], big.info["adjoint_order"], big.info["adjoint_blocks_per_cu"]) == (
        64, mlbm.MLBM_ORDER_XCD_RANGE, 2)
    h32 = mlbm.mlbm_create(9, (512, 512, 1), 0.8, 1.0, mlbm.MLBM_STORE_F32)
    i = h32.info
    assert (i["adjoint_form"], i["adjoint_block_x"], i["adjoint_order"], i["adjoint_blocks_per_cu"]) == (
        mlbm.MLBM_ADJ_CHANNEL, 64, mlbm.MLBM_ORDER_INTERLEAVE8, 0)
    assert i["adjoint_temporal_stores"] == 1
    h64 = mlbm.mlbm_create(9, (512, 512, 1), 0.8, 1.0, mlbm.MLBM_STORE_F64)    # F64 below 2^20 cells: per-XCD rows
    assert h64.info["adjoint_order"] == mlbm.MLBM_ORDER_XCD_RANGE
    h64b = mlbm.mlbm_create(9, (1024, 1024, 1), 0.8, 1.0, mlbm.MLBM_STORE_F64)
    assert h64b.info["adjoint_order"] == mlbm.MLBM_ORDER_INTERLEAVE8
    mlbm.mlbm_set_adjoint_launch(h, mlbm.MLBM_ADJ_CHANNEL, 128, mlbm.MLBM_ORDER_NATURAL, 3, 1)
    i = h.info
    assert (i["adjoint_block_x"], i["adjoint_order"], i["adjoint_blocks_per_cu"], i["adjoint_temporal_stores"]) == (
        128, mlbm.MLBM_ORDER_NATURAL, 3, 1)
    mlbm.mlbm_set_adjoint_launch(h, mlbm.MLBM_ADJ_CELL)
    assert h.info["adjoint_form"] == mlbm.MLBM_ADJ_CELL and h.info["adjoint_block_x"] == 0
    mlbm.mlbm_set_adjoint_launch(h)
    mlbm.mlbm_set_magnetic_field(h, [0.0, 0.1, 0.0])
    assert h.info["adjoint_form"] == mlbm.MLBM_ADJ_CELL       # the field runs in the cell form only
    for bad in ((3, 0, -1, -1, -1), (0, 96, -1, -1, -1), (0, 0, 3, -1, -1), (0, 0, -1, 33, -1), (0, 0, -1, -1, 2)):
        with pytest.raises(mlbm.MlbmError) as e:
            mlbm.mlbm_set_adjoint_launch(h, *bad)
        assert e.value.code == mlbm.MLBM_EINVAL


def test_one_hip_runtime_whatever_the_import_order():
    """The binding loads the library after torch, so the library binds to the HIP
    runtime torch already holds (torch ships it under another file name with the
    same soname).  A second runtime in the process finds no device once the
    first one has started.  Checked in fresh processes through the mapped files."""
    import subprocess
    import sys
    probe = (
        "import os, sys\n"
        "sys.path.insert(0, {root!r})\n"
        "{first}\n{second}\n"
        "maps = open('/proc/self/maps').read().split('\\n')\n"
        "paths = {{l.split()[-1] for l in maps if 'libamdhip64' in l}}\n"
        "print(len(paths))\n"
    )
    lib_first = "from paper_1309_1656_amd import mlbm; mlbm.load_library()"
    torch_first = "import torch"
    for first, second in ((lib_first, torch_first), (torch_first, lib_first)):
        out = subprocess.run([sys.executable, "-c", probe.format(root=ROOT, first=first, second=second)],
                             capture_output=True, text=True, timeout=300)
        assert out.returncode == 0, out.stderr
        assert out.stdout.strip().splitlines()[-1] == "1", (first, out.stdout)
