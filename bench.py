"""Benchmark of the matrix-valued quantum lattice Boltzmann step on one GPU.

Default workload: D3Q19, 128^3 periodic cells, tau = 0.8, beta0 = 1, seeded
smooth Fermi-Dirac initial state (paper_1309_1656_amd.synthetic), K = 500
steps.  A "step" is one time step of the method (moments, polynomial
equilibrium, BGK collision, streaming) over the whole lattice; the timed
region is one mlbm_step(K) call with its inputs resident in device memory.

Printed: one JSON line.  `value` is MLUPS (10^6 cell updates per second) of
the double-precision step.  Also reported: FP32 and FP16 scaled-deviation
storage on the same workload, the fused kernel's average duration and HBM
roofline fraction, the forward + adjoint time of the differentiable rollout
(D2Q9 512^2, FP32, 200 steps, checkpoints every 20) next to the plain FP64
forward, one D3Q19 128^3 adjoint step in FP64 and FP32, the magnetic-field
and variant steps, the launch-bound Riemann run eager and as a HIP graph, the
library's plain device copy (the achievable-bandwidth reference), the error
against the stored FP64 oracle run, and the CPU oracle on the headline
workload (D3Q19 128^3, a few timed steps) and on the smaller workloads.

With --sweep the line also carries "sweep": every step workload (D2Q9 64^2,
512^2, 1024^2 shear; D3Q19 64^3, 128^3, 384^3) in each storage type it is
run in, with the automatic launch shape.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
       [--storage f64|fp32|f16dev] [--skip-extras] [--no-cpu-baseline] [--sweep]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, AMD published peak
TRAFFIC_FILES = {"f64": os.path.join(ROOT, "profiles", "k_step_d3q19_128_traffic.json"),
                 "fp32": os.path.join(ROOT, "profiles", "k_step_d3q19_128_fp32_traffic.json"),
                 "f16dev": os.path.join(ROOT, "profiles", "k_step_d3q19_128_f16dev_traffic.json")}
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1309_1656_amd", "csrc", f) for f in ("step.hip", "common.hpp", "block_order.hpp")]


# step workloads (names in paper_1309_1656_amd.synthetic.WORKLOADS) and the storage types the sweep runs them in
STEP_WORKLOADS = {"d2q9_64": ("f64",), "d2q9_512_adjoint": ("f64", "fp32"), "d2q9_1024_shear": ("f64", "fp32"),
                  "d3q19_64": ("f64", "fp32", "f16dev"), "d3q19_128": ("f64", "fp32", "f16dev"),
                  "d3q19_384": ("f64", "fp32", "f16dev")}
STORAGE_NAMES = ("f64", "fp32", "f16dev")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="d3q19_128", choices=sorted(STEP_WORKLOADS))
    ap.add_argument("--skip-extras", action="store_true", help="only the headline measurement")
    ap.add_argument("--storage", choices=("f64", "fp32", "f16dev"), default="f64",
                    help="storage type of the headline measurement (f64 is the benchmark; the others serve "
                         "per-precision profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--adjoint-step", action="store_true",
                    help="measure the D3Q19 128^3 adjoint step also with --skip-extras (for counter runs)")
    ap.add_argument("--sweep", action="store_true",
                    help="also measure every step workload in each storage type it is run in")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 1 GiB device copy (reference for hardware byte counters)")
    return ap.parse_args()


def device_inputs(h, f):
    import torch
    rho4 = np.concatenate([f["trrho"][None], f["r"]])
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    return to(rho4), to(h.info["xi"] * f["u_lat"]), to(f["T"])


def dims_of(shape):
    return (shape[1], shape[0], 1) if len(shape) == 2 else (shape[2], shape[1], shape[0])


def time_region(fn, reps=1):
    """Average milliseconds of fn() over reps, by events on the current stream."""
    import torch
    s = torch.cuda.current_stream()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(reps):
        fn()
    b.record(s)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def measure_step(shape, seed, tau, storage, steps, warmup, f, field=None, isothermal=False, positivity=False):
    """MLUPS of mlbm_step(steps) and the fused kernel's average duration.

    field: None, "uniform" (one mu B for the grid) or "map" (mu B per cell,
    read by every step: 24 more bytes per cell)."""
    import torch
    from paper_1309_1656_amd import mlbm
    Q = 9 if len(shape) == 2 else 19
    h = mlbm.mlbm_create(Q, dims_of(shape), tau, 1.0, storage)
    W = h.empty_field()
    mlbm.mlbm_init_equilibrium(h, W, *device_inputs(h, f))
    extra_bytes = 0
    if isothermal:
        mlbm.mlbm_set_eq_mode(h, mlbm.MLBM_EQ_ISOTHERMAL)
    if positivity:
        mlbm.mlbm_set_positivity(h, 1)
    if field == "uniform":
        mlbm.mlbm_set_magnetic_field(h, [0.01, -0.02, 0.03])
    elif field == "map":
        rng = np.random.default_rng(seed + 7)
        bmap = torch.from_numpy(rng.normal(0, 0.02, size=(3,) + tuple(shape))).cuda()
        mlbm.mlbm_set_magnetic_field_map(h, bmap)
        extra_bytes = 3 * 8
    scratch = h.empty_field()
    g0, _ = mlbm.mlbm_moments(h, W)
    if warmup:
        mlbm.mlbm_step(h, W, scratch, warmup)
    torch.cuda.synchronize()
    t_all = time_region(lambda: mlbm.mlbm_step(h, W, scratch, steps))
    # mlbm_step(n >= 2) is the collide-only pass, n - 2 fused passes and the pass that collides and
    # pushes into W, so two calls differ by fused passes alone: the fused pass is
    # (t(steps) - t(2)) / (steps - 2)
    t_base = time_region(lambda: mlbm.mlbm_step(h, W, scratch, 2), reps=5)
    g1, nneg = mlbm.mlbm_moments(h, W)
    N = int(np.prod(shape))
    fused_ms = (t_all - t_base) / (steps - 2)
    bytes_per_cell = 2 * 4 * Q * {0: 8, 1: 4, 2: 2}[storage] + extra_bytes
    achieved = bytes_per_cell * N / (fused_ms * 1e-3) / 1e9
    drift = float(np.max(np.abs(g1 - g0)) / np.max(np.abs(g0)))
    info = h.info
    out = {
        "launch": {"block_x": info["launch_block_x"], "order": ["natural", "xcd_range", "interleave8"][info["launch_order"]],
                   "blocks_per_cu": info["launch_blocks_per_cu"], "temporal_stores": info["launch_temporal_stores"]},
        "mlups": N * steps / (t_all * 1e-3) / 1e6,
        "ms_per_step": t_all / steps,
        "fused_kernel_ms": fused_ms,
        "fused_kernel_GBps": achieved,
        "hbm_frac": achieved / HBM_PEAK_GBS,
        "bytes_per_cell": bytes_per_cell,
        "global_drift_rel": drift,
        "n_neg_eig": nneg,
    }
    h.destroy()
    return out


def workload_fields(name):
    """Seeded macroscopic input fields of a step workload."""
    from paper_1309_1656_amd import synthetic
    wl = synthetic.WORKLOADS[name]
    if name == "d2q9_1024_shear":
        return synthetic.shear_band_fields(wl["shape"], wl["seed"])
    return synthetic.macroscopic_fields(wl["shape"], wl["seed"])


def sweep(warmup):
    """Every step workload in each storage type it is run in (steps: the
    workload's own, at most 200 above 5e7 cells)."""
    import torch
    from paper_1309_1656_amd import synthetic
    rows = []
    for name, storages in STEP_WORKLOADS.items():
        wl = synthetic.WORKLOADS[name]
        shape = wl["shape"]
        f = workload_fields(name)
        steps = min(wl["steps"], 200) if np.prod(shape) > 5e7 else wl["steps"]
        for st in storages:
            log(f"sweep: {name} {st}, {steps} steps")
            r = measure_step(shape, wl["seed"], wl["tau"], STORAGE_NAMES.index(st), steps, warmup, f)
            log(f"  {r['mlups']:.0f} MLUPS, fused {r['fused_kernel_GBps']:.0f} GB/s")
            rows.append({"workload": name, "grid": list(reversed(shape)), "tau": wl["tau"], "storage": st,
                         "steps": steps, "mlups": r["mlups"], "fused_kernel_ms": r["fused_kernel_ms"],
                         "fused_kernel_GBps": r["fused_kernel_GBps"], "hbm_frac": r["hbm_frac"],
                         "launch": r["launch"]})
            torch.cuda.empty_cache()
    return rows


def measure_adjoint(warmup):
    """Forward + adjoint rollout (D2Q9 512^2, FP32, 200 steps, K = 20) vs the plain FP32 and FP64 forward
    of the same grid and steps."""
    import torch
    from paper_1309_1656_amd import mlbm, synthetic
    from paper_1309_1656_amd.rollout import MLBMRollout
    wl = synthetic.WORKLOADS["d2q9_512_adjoint"]
    shape, steps, tau = wl["shape"], wl["steps"], wl["tau"]
    f = synthetic.macroscopic_fields(shape, wl["seed"])
    rt = torch.from_numpy(synthetic.target_bloch_field(shape, wl["seed"] + 100)).cuda()
    h32 = mlbm.mlbm_create(9, dims_of(shape), tau, 1.0, mlbm.MLBM_STORE_F32)
    W0 = h32.empty_field()
    mlbm.mlbm_init_equilibrium(h32, W0, *device_inputs(h32, f))
    W0.requires_grad_(True)
    tau_t = torch.tensor(tau, dtype=torch.float64, requires_grad=True)

    def fwd_bwd():
        W0.grad = None
        tau_t.grad = None
        loss = MLBMRollout.apply(W0, tau_t, h32, steps, 20, rt)
        loss.backward()
        return loss

    for _ in range(max(2, warmup // 5)):
        fwd_bwd()
    t_fb = time_region(fwd_bwd, reps=5)
    # the two halves of one more run, by events on the current stream
    s = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    W0.grad = None
    tau_t.grad = None
    torch.cuda.synchronize()
    ev[0].record(s)
    loss = MLBMRollout.apply(W0, tau_t, h32, steps, 20, rt)
    ev[1].record(s)
    loss.backward()
    ev[2].record(s)
    torch.cuda.synchronize()
    t_fwd_part, t_bwd_part = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    W32 = W0.detach().clone()
    s32 = h32.empty_field()
    mlbm.mlbm_step(h32, W32, s32, 20)
    t_f32 = time_region(lambda: mlbm.mlbm_step(h32, W32, s32, steps), reps=5)
    h64 = mlbm.mlbm_create(9, dims_of(shape), tau, 1.0, mlbm.MLBM_STORE_F64)
    W64 = h64.empty_field()
    mlbm.mlbm_init_equilibrium(h64, W64, *device_inputs(h64, f))
    s64 = h64.empty_field()
    mlbm.mlbm_step(h64, W64, s64, 20)
    t_f64 = time_region(lambda: mlbm.mlbm_step(h64, W64, s64, steps), reps=3)
    return {"workload": "d2q9_512^2_f32_200steps_ckpt20", "fwd_adjoint_ms": t_fb,
            "forward_part_ms": t_fwd_part, "backward_part_ms": t_bwd_part,
            "plain_f32_forward_ms": t_f32, "ratio_to_f32_forward": t_fb / t_f32,
            "plain_f64_forward_ms": t_f64, "ratio_to_f64_forward": t_fb / t_f64,
            "grad_tau": float(tau_t.grad), "grad_W0_norm": float(W0.grad.norm())}


def measure_adjoint_step(shape, tau, f, storage, reps=10):
    """One mlbm_adjoint_step (W_n as stored, lam_{n+1} pulled, dL/domega finalised) on a 3-D workload:
    average ms and the rate of its algorithmic bytes (read W_n and lam_{n+1}, write lam_n: 3 4 Q s per cell)."""
    import torch
    from paper_1309_1656_amd import mlbm
    Q = 19
    h = mlbm.mlbm_create(Q, dims_of(shape), tau, 1.0, storage)
    W = h.empty_field()
    mlbm.mlbm_init_equilibrium(h, W, *device_inputs(h, f))
    gen = torch.Generator(device="cuda").manual_seed(11)
    lam1 = torch.randn(h.field_shape, dtype=h.field_dtype, device="cuda", generator=gen)
    lam0 = h.empty_field()
    dom = torch.zeros(1, dtype=torch.float64, device="cuda")
    mlbm.mlbm_adjoint_step(h, W, lam1, lam0, dom)
    t = time_region(lambda: mlbm.mlbm_adjoint_step(h, W, lam1, lam0, dom), reps=reps)
    N = int(np.prod(shape))
    by = 3 * 4 * Q * {0: 8, 1: 4}[storage] * N
    h.destroy()
    return {"ms": t, "GBps": by / (t * 1e-3) / 1e9, "hbm_frac": by / (t * 1e-3) / 1e9 / HBM_PEAK_GBS}


GOLDEN_128 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                          "oracle_d3q19_128_tau0.8_500.npz")


def f16dev_decode(h, vals):
    """Decoded populations of F16 scaled-deviation values [4, Q, ...] (the storage format of
    include/mlbm.h: a = R_ki + s_i h, s_i the power of two nearest w_i S, summed in float)."""
    info = h.info
    x = np.log2(np.asarray(info["w"]) * info["f16_scale"])
    sc = np.ldexp(1.0, (np.sign(x) * np.floor(np.abs(x) + 0.5)).astype(np.int64)).astype(np.float32)
    extra = vals.ndim - 2
    ref = np.asarray(info["f16_ref"], dtype=np.float32).reshape((4, -1) + (1,) * extra)
    return (ref + sc.reshape((1, -1) + (1,) * extra) * vals.astype(np.float32)).astype(np.float64)


def measure_accuracy(f, storage):
    """Error of the benchmark workload (D3Q19 128^3, tau 0.8, 500 steps from the
    same initial state) against the stored FP64 oracle run: normwise over the
    1 024 stored cells, max over Pauli components of max|d a_k| / max|a_k|.
    F16 deviation storage is compared population by population (decoded) and
    on the cell density matrices."""
    import torch
    from paper_1309_1656_amd import mlbm
    if not os.path.exists(GOLDEN_128):
        return None
    g = np.load(GOLDEN_128)
    shape = (128, 128, 128)
    h = mlbm.mlbm_create(19, dims_of(shape), float(g["meta"][0]), float(g["meta"][2]), storage)
    W = h.empty_field()
    mlbm.mlbm_init_equilibrium(h, W, *device_inputs(h, f))
    mlbm.mlbm_step(h, W, h.empty_field(), int(g["meta"][1]))
    idx = tuple(torch.from_numpy(c).cuda() for c in np.unravel_index(g["cells"], shape))
    sel = h.pauli_view(W)[(slice(None), slice(None)) + idx]
    if storage == mlbm.MLBM_STORE_F16DEV:
        got = f16dev_decode(h, sel.cpu().numpy())
        pop = max(float(np.abs(got[k] - g["values"][k]).max() / g["maxabs"][k]) for k in range(4))
        rho4 = torch.empty((4,) + shape, dtype=torch.float64, device="cuda")
        mlbm.mlbm_moments(h, W, rho4=rho4)
        got_rho = rho4[(slice(None),) + idx].cpu().numpy()
        ref = g["values"].sum(axis=1)
        rho = max(float(np.abs(got_rho[k] - ref[k]).max() / np.abs(ref[k]).max()) for k in range(4))
        err = {"populations": pop, "rho": rho}
    else:
        got = sel.to(torch.float64).cpu().numpy()
        err = max(float(np.abs(got[k] - g["values"][k]).max() / g["maxabs"][k]) for k in range(4))
    h.destroy()
    return err


def measure_launch_bound():
    """The Riemann workload (D2Q9 2048 x 2, 385 steps): one mlbm_step call
    launched eagerly against the same call captured once in a HIP graph."""
    import torch
    from paper_1309_1656_amd import mlbm, synthetic
    wl = synthetic.WORKLOADS["d2q9_riemann"]
    f = synthetic.riemann_fields(wl["shape"])
    h = mlbm.mlbm_create(9, dims_of(wl["shape"]), wl["tau"], 1.0, mlbm.MLBM_STORE_F64)
    W = h.empty_field()
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    mlbm.mlbm_init_chemical(h, W, to(f["nu"]), to(h.info["xi"] * f["u_lat"]), to(f["T"]))
    tmp = h.empty_field()
    n = wl["steps"]
    mlbm.mlbm_step(h, W, tmp, 5)
    t_eager = time_region(lambda: mlbm.mlbm_step(h, W, tmp, n), reps=3)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        mlbm.mlbm_step(h, W, tmp, 2)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        mlbm.mlbm_step(h, W, tmp, n)
    g.replay()
    t_graph = time_region(g.replay, reps=3)
    N = int(np.prod(wl["shape"]))
    return {"workload": "D2Q9 2048x2 Riemann problem, 385 steps, FP64", "eager_ms": t_eager, "graph_ms": t_graph,
            "eager_mlups": N * n / (t_eager * 1e-3) / 1e6, "graph_mlups": N * n / (t_graph * 1e-3) / 1e6}


def copy_bandwidth():
    """Plain device copies of 2 GiB each way: the library's 16-byte-per-thread
    streaming copy (the achievable-bandwidth reference) and torch's copy_."""
    import torch
    from paper_1309_1656_amd import mlbm
    n = 1 << 28   # float64 elements
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    mlbm.mlbm_device_copy(a, b)
    ms = time_region(lambda: mlbm.mlbm_device_copy(a, b), reps=10)
    b.copy_(a)
    ms_torch = time_region(lambda: b.copy_(a), reps=5)
    del a, b
    return {"GBps": 2 * n * 8 / (ms * 1e-3) / 1e9, "torch_copy_GBps": 2 * n * 8 / (ms_torch * 1e-3) / 1e9}


def kernel_source_hash():
    """sha256 of the step kernel's code (comments and blank lines removed, so
    that a comment edit does not invalidate the stored counter readings)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update("\n".join(ln.rstrip() for ln in text.splitlines() if ln.strip()).encode())
    return h.hexdigest()


def measured_traffic(storage="f64"):
    """HBM bytes per fused-kernel launch from the stored counter summary, if it matches the current kernel."""
    path = TRAFFIC_FILES[storage]
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return t["hbm_bytes_per_launch"]


def copy_probe():
    import torch
    n = (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()


def _oracle_rate(lat, f, tau, min_steps, seconds):
    from oracle import qlbm
    W = qlbm.init_equilibrium(lat, f["trrho"], f["r"], lat.xi * f["u_lat"], f["T"])
    W = qlbm.step(lat, W, tau)           # warm-up
    n, t0 = 0, time.perf_counter()
    while n < min_steps or time.perf_counter() - t0 < seconds:
        W = qlbm.step(lat, W, tau)
        n += 1
    dt = time.perf_counter() - t0
    return int(np.prod(f["T"].shape)) * n / dt / 1e6, n


def cpu_baseline(seconds=10.0):
    """The FP64 oracle on the headline workload: D3Q19 128^3, tau 0.8, the same
    seeded initial state, one warm-up step, then at least 3 timed steps (and at
    least `seconds`); also its rate on the smaller step workloads (a few steps
    each) and on a D3Q19 48^3 sample of the same initial-state family."""
    from threadpoolctl import threadpool_limits
    from oracle import qlbm
    from paper_1309_1656_amd import synthetic
    wl = synthetic.WORKLOADS["d3q19_128"]
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):    # the oracle is elementwise NumPy; hold any library pool to one thread
        rate, n = _oracle_rate(qlbm.Lattice(3), workload_fields("d3q19_128"), wl["tau"], 3, seconds)
        per = {}
        for name, lat_d, steps in (("d2q9_64", 2, 20), ("d2q9_1024_shear", 2, 2), ("d3q19_64", 3, 3)):
            w = synthetic.WORKLOADS[name]
            per[name] = {"MLUPS": _oracle_rate(qlbm.Lattice(lat_d), workload_fields(name), w["tau"], steps, 0.0)[0],
                         "steps": steps}
        shape48 = (48, 48, 48)
        per["d3q19_48_sample"] = {
            "MLUPS": _oracle_rate(qlbm.Lattice(3), synthetic.macroscopic_fields(shape48, synthetic.BASE_SEED + 3), 0.8,
                                  3, 0.0)[0], "steps": 3}
    return {"value": rate, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"D3Q19 128^3 cells (the headline workload: same seeded initial state, tau {wl['tau']}), "
                      f"1 warm-up step then {n} timed steps; NumPy elementwise work, one thread",
            "per_workload": per, "wall_s": time.perf_counter() - t0,
            "host_cpus": os.cpu_count(), "host_cpu_model": _cpu_model()}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(spatial sharding by slabs is designed, not built)", file=sys.stderr)
        sys.exit(2)
    if args.steps < 3:
        print("--steps must be at least 3: the fused pass is timed as the difference of mlbm_step(steps) and "
              "mlbm_step(2)", file=sys.stderr)
        sys.exit(2)
    # The CPU oracle leg runs in a child process of its own (one host core, started before this
    # process touches the GPU), beside the GPU measurements instead of after them.
    cpu_job = None
    if not args.no_cpu_baseline:
        import concurrent.futures
        import multiprocessing
        cpu_pool = concurrent.futures.ProcessPoolExecutor(max_workers=1, mp_context=multiprocessing.get_context("spawn"))
        cpu_job = cpu_pool.submit(cpu_baseline)
    import torch
    from paper_1309_1656_amd import mlbm, synthetic
    torch.cuda.set_device(0)
    mlbm.load_library()
    wl = synthetic.WORKLOADS[args.workload]
    shape, tau = wl["shape"], wl["tau"]
    log(f"workload {args.workload} {shape} tau={tau}: generating inputs")
    f = workload_fields(args.workload)
    storage = {"f64": mlbm.MLBM_STORE_F64, "fp32": mlbm.MLBM_STORE_F32, "f16dev": mlbm.MLBM_STORE_F16DEV}[args.storage]
    log(f"{args.storage} step")
    r64 = measure_step(shape, wl["seed"], tau, storage, args.steps, args.warmup, f)
    log(f"  {r64['mlups']:.0f} MLUPS, fused {r64['fused_kernel_ms']:.4f} ms, {r64['fused_kernel_GBps']:.0f} GB/s")
    copy = copy_bandwidth()
    log(f"  device copy {copy['GBps']:.0f} GB/s (torch copy_ {copy['torch_copy_GBps']:.0f} GB/s)")
    extras = {}
    if not args.skip_extras:
        for name, st in (("fp32", mlbm.MLBM_STORE_F32), ("f16dev", mlbm.MLBM_STORE_F16DEV)):
            if name == args.storage:
                continue
            log(f"{name} step")
            extras[name] = measure_step(shape, wl["seed"], tau, st, args.steps, args.warmup, f)
            log(f"  {extras[name]['mlups']:.0f} MLUPS, {extras[name]['fused_kernel_GBps']:.0f} GB/s")
        extras["magnetic_f64"] = {}
        for kind in ("uniform", "map"):
            log(f"FP64 step with a {kind} magnetic field")
            extras["magnetic_f64"][kind] = measure_step(shape, wl["seed"], tau, mlbm.MLBM_STORE_F64, args.steps,
                                                        args.warmup, f, field=kind)
            log(f"  {extras['magnetic_f64'][kind]['mlups']:.0f} MLUPS, "
                f"{extras['magnetic_f64'][kind]['fused_kernel_GBps']:.0f} GB/s")
        extras["variants_f64"] = {}
        for name, kw in (("isothermal", dict(isothermal=True)), ("positivity", dict(positivity=True)),
                         ("isothermal_positivity", dict(isothermal=True, positivity=True))):
            log(f"FP64 step, {name} variant")
            extras["variants_f64"][name] = measure_step(shape, wl["seed"], tau, mlbm.MLBM_STORE_F64, args.steps,
                                                        args.warmup, f, **kw)
            log(f"  {extras['variants_f64'][name]['mlups']:.0f} MLUPS, "
                f"{extras['variants_f64'][name]['fused_kernel_GBps']:.0f} GB/s")
        log("launch-bound Riemann workload, eager and graph")
        extras["launch_bound"] = measure_launch_bound()
        log(f"  eager {extras['launch_bound']['eager_ms']:.3f} ms, graph {extras['launch_bound']['graph_ms']:.3f} ms")
        log("forward + adjoint rollout")
        extras["adjoint"] = measure_adjoint(args.warmup)
        log(f"  {extras['adjoint']['fwd_adjoint_ms']:.2f} ms: {extras['adjoint']['ratio_to_f32_forward']:.2f}x the FP32 "
            f"forward, {extras['adjoint']['ratio_to_f64_forward']:.2f}x the FP64 forward")
    if args.workload == "d3q19_128" and (args.adjoint_step or not args.skip_extras):
        log("adjoint step, D3Q19 128^3")
        adj3 = {"workload": "D3Q19 128^3, one mlbm_adjoint_step", "f64_fused_forward_ms": r64["fused_kernel_ms"]}
        for name, st in (("f64", mlbm.MLBM_STORE_F64), ("fp32", mlbm.MLBM_STORE_F32)):
            adj3[name] = measure_adjoint_step(shape, tau, f, st)
            adj3[name]["ratio_to_f64_forward_pass"] = adj3[name]["ms"] / r64["fused_kernel_ms"]
            log(f"  {name}: {adj3[name]['ms'] * 1e3:.1f} us, {adj3[name]['GBps']:.0f} GB/s")
        extras.setdefault("adjoint", {})["d3q19_128_step"] = adj3
    if args.sweep:
        extras["sweep"] = sweep(args.warmup)
    if args.workload == "d3q19_128" and not args.skip_extras:
        log("accuracy against the stored FP64 oracle run")
        acc = {"reference": "FP64 oracle, same initial state, tau 0.8, 500 steps; 1024 stored cells; "
                            "max over Pauli components k of max|d a_k| / max|a_k| (FP16: of the decoded "
                            "populations and of the cell density matrices)"}
        for name, st in (("f64", mlbm.MLBM_STORE_F64), ("fp32", mlbm.MLBM_STORE_F32),
                         ("f16dev", mlbm.MLBM_STORE_F16DEV)):
            acc[name] = measure_accuracy(f, st)
        extras["accuracy_vs_oracle"] = acc
        log(f"  {acc}")
    Q = 9 if len(shape) == 2 else 19
    grid = "x".join(str(s) for s in reversed(shape))
    line = {
        "metric": "MLUPS & HBM-roofline fraction, D3Q19 step: FP32 vs FP64, fwd+adjoint time",
        "value": r64["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {"workload": f"{'D2Q9' if Q == 9 else 'D3Q19'} {grid} periodic, tau {tau}, beta0 1, "
                               f"smooth Fermi-Dirac initial state, {args.storage.upper()} storage",
                   "lattice": "D2Q9" if Q == 9 else "D3Q19", "grid": list(reversed(shape)), "tau": tau},
        "roofline": {"bound": "hbm", "achieved": r64["fused_kernel_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": r64["fused_kernel_GBps"] / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.storage) if args.workload == "d3q19_128" else None,
                     "algorithmic_bytes_per_launch": r64["bytes_per_cell"] * int(np.prod(shape)),
                     "kernel": f"k_step<{Q}, {args.storage.upper()}, pull, collide>", "kernel_ms": r64["fused_kernel_ms"],
                     "launch": r64["launch"],
                     "bytes_per_cell": r64["bytes_per_cell"],
                     "device_copy_GBps": copy["GBps"], "frac_of_device_copy": r64["fused_kernel_GBps"] / copy["GBps"],
                     "torch_copy_GBps": copy["torch_copy_GBps"]},
        args.storage: r64,
    }
    line.update(extras)
    if cpu_job is not None:
        log("CPU oracle baseline (waiting for the child process)")
        try:
            line["cpu_baseline"] = cpu_job.result()
        except Exception as e:          # the child could not run (e.g. a launcher that forbids it): run it here
            log(f"  child process failed ({type(e).__name__}: {e}); timing the oracle in this process")
            line["cpu_baseline"] = cpu_baseline()
        cpu_pool.shutdown()
        log(f"  {line['cpu_baseline']['value']:.3f} MLUPS")
    if args.copy_probe:
        copy_probe()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
