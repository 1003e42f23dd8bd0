"""Benchmark of the fused QPINN circuit step on one MI355X.

A step is one fused Maxwell evaluation over the whole point set: gate table, per-point forward
with three input tangents, readout, residual loss, adjoint sweep with uncompute, and the FP64
gradient/loss reductions.  Default workload: 12 qubits, 8 layers of RX/RY/RZ + CNOT ring,
262144 collocation points (the 64^3 grid size of the paper's training set), complex64.

Prints ONE JSON line on stdout.  Extra legs (on by default, short):
  * cpu_baseline - the CPU oracle timed on a bounded sample of the same points;
  * plain_gpu    - the plain per-gate + finite-difference path on the same GPU, timed on a
                   point subset and a parameter subset, extrapolated to the full step;
  * parity       - outputs and tangents of sampled points of the timed run vs the oracle.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X published FP32 peak, dense matrix cores (and the vector ALU's)
PROFILES = os.path.join(ROOT, "profiles")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def flops_per_point(n_fused: int, n: int) -> float:
    """Algorithmic FP32 work of one point, in the FMA-slot count used for the roofline:
    16 flop per amplitude per statevector for one fused 2x2 gate (8 FMA-slot operations, 4 per
    real part of the complex 2x2 row), applied to 4 statevectors in the forward (psi and three
    tangents) and 8 in the adjoint (uncompute + pull-back), plus the per-gate adjoint products
    counted as 4 statevector-equivalents: (4 + 8 + 4) x 16 = 256 flop per amplitude per gate.
    Encoding, readout, seeds and the LDS exchanges are not counted."""
    return float(n_fused) * (2 ** n) * 256


def executed_flops_per_point(n_fused: int, n: int, n_folded: int = 0) -> float:
    """Flops the kernel's algorithm needs for the same work with mul = 1 and fma = 2: 14 per
    amplitude per statevector and gate (1 mul + 3 fma per real part), and the gate statistic
    S_k = Im <lambda|sigma_k|psi> at 4 statevector pairs x 3 components x 4 fma x 2 = 96 per
    amplitude pair, 48 per amplitude: (4 x 14 + 8 x 14 + 48) = 216 per amplitude per gate.  The n_folded gates of
    an opening rotation stage are folded into the product-state encoding: they are neither applied
    nor pulled back (only their statistic, 48, remains)."""
    return (2 ** n) * (float(n_fused) * 216 - float(n_folded) * 168)


def matrix_core_share(n_fused: int, n_folded: int = 0) -> float:
    """Share of executed_flops_per_point done on the matrix cores: the 2x2 gate products (12 x 14
    per amplitude per applied gate) run as v_mfma_f32_4x4x1f32, the gate statistics (48) on the
    vector ALU."""
    total = float(n_fused) * 216 - float(n_folded) * 168
    return 168.0 * (n_fused - n_folded) / total if total > 0 else 0.0


# Sources that determine each kernel's code and memory accesses (device code and the planner
# that writes its plan image).  A counter record taken for one digest does not describe a kernel
# built from other sources.
KERNEL_SOURCES = {
    "k_fused": ["fused_kernel.hpp", "fused.hip", "fused.hpp", "fused_n*.hip", "qp_internal.hpp", "grads_dev.hpp",
                "rot_dev.hpp", "plan.cpp", "plan.hpp"],
    "k_batch": ["batch.hip", "batch_ph.hip", "batch_kernel.hpp", "batch.hpp", "batch_api.cpp", "fused_kernel.hpp",
                "fused.hpp", "qp_internal.hpp", "grads_dev.hpp", "rot_dev.hpp", "plan.cpp", "plan.hpp"],
}


def sources_digest(kernel: str = "k_fused") -> str:
    """SHA-256 of the sources behind `kernel` (KERNEL_SOURCES)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    files = []
    for pat in KERNEL_SOURCES[kernel]:
        files += glob.glob(os.path.join(ROOT, "paper_2506_23246_amd", "csrc", pat))
    for f in sorted(set(files)):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed counter summaries under
    profiles/ (FETCH_SIZE and WRITE_SIZE scaled by a copy kernel's readings), or None when there
    is no record for the current sources."""
    import glob
    digest = sources_digest(kernel)
    for path in sorted(glob.glob(os.path.join(PROFILES, "*hbm_counters*.md"))):
        with open(path) as fh:
            for ln in fh:
                ln = ln.strip()
                if not ln.startswith("{") or '"traffic_bytes_per_launch"' not in ln:
                    continue
                try:
                    rec = json.loads(ln)
                except ValueError:
                    continue
                if rec.get("kernel") == kernel and rec.get("workload") == workload and rec.get("sources_sha256") == digest:
                    return rec["traffic_bytes_per_launch"], os.path.relpath(path, ROOT)
    return None, None


def cpu_baseline(w, sample_points: int | None = None):
    """The CPU oracle (complex128, explicit Kronecker-product operators, stored-state reverse mode)
    timed on this host's cores: the same three phases as a full evaluation (forward with tangents
    per point chunk, loss seeds over the sample, reverse mode per chunk), spread over a process
    pool of one single-threaded worker per core.  Runs before the process touches the GPU (the
    pool forks)."""
    from oracle import parallel as OP
    n = w.circuit.n
    workers = OP.host_cores()
    chunk = OP.default_chunk(n)
    if sample_points is None:   # about 10-30 s of work: two chunks per worker at 12 qubits
        sample_points = min(len(w.points), workers * chunk * (2 if n >= 12 else 8))
    pts = w.points[:sample_points]
    with OP.Pool(workers) as pool:
        OP.simulate(pool, w.circuit, w.params, pts[:workers], chunk=1)     # start the workers
        t0 = time.perf_counter()
        OP.maxwell_eval(pool, w.circuit, w.params, pts, w.loss, chunk=chunk)
        dt = time.perf_counter() - t0
    try:
        from threadpoolctl import threadpool_info
        blas = sorted({f"{d.get('internal_api')}:{d.get('num_threads')}" for d in threadpool_info()})
    except Exception:  # pragma: no cover
        blas = []
    rate = sample_points / dt
    return {"value": round(rate, 3), "unit": "evals/s", "cores": workers, "kind": "oracle",
            "nproc": os.cpu_count(), "blas_threads_per_worker": 1, "blas_in_parent": blas,
            "sample": f"first {sample_points} points of the same workload in chunks of {chunk} over {workers} "
                      f"single-threaded worker processes: complex128 Kronecker-product forward with 3 tangents, "
                      f"Maxwell loss seeds, stored-state reverse-mode gradient; {dt:.1f} s wall",
            "full_step_s_extrapolated": round(len(w.points) / rate, 1)}


def c1_plain_fp64(ctx, dev, reps: int = 20):
    """Wall time of the plain FP64 method on its 4-qubit, 2-layer workload (1024 points): one
    kernel per gate on an HBM statevector batch, readout, input tangents by central finite
    differences (7 forwards).  Launch-latency bound; reported as wall time per evaluation."""
    import torch
    import workloads as W
    from paper_2506_23246_amd.api import Circuit
    w = W.config(0)
    c = Circuit(ctx, w.circuit)
    prm = torch.tensor(w.params, device=dev)
    pts = torch.tensor(w.points, device=dev)
    c.plain_eval(prm, pts, precision=64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        c.plain_eval(prm, pts, precision=64)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    launches = len(w.circuit.gates) * 7
    c.close()
    return {"workload": w.name, "points": len(w.points), "wall_ms": round(dt * 1e3, 4),
            "evals_per_s": round(len(w.points) / dt, 1),
            "what": f"FP64 complex statevectors, one kernel per gate ({launches} gate launches: forward + 6 "
                    f"central-FD forwards, h = 1e-5), eager, mean of {reps} calls"}


def parity_vs_stored_oracle(ctx, w, name):
    """The fused step at the default launch on a stored oracle set (tests/golden): normwise relative
    errors of outputs, tangents (at the stored indices), loss and gradient (over the whole set)."""
    import numpy as np
    from paper_2506_23246_amd.api import Circuit
    from tests.golden.make_oracle_fixtures import SETS, load
    ref = load(name)
    ws = SETS[name]()
    c = Circuit(ctx, ws.circuit)
    r = c.maxwell(ws.params, ws.points, ws.loss)
    idx = ref["idx"]

    def rel(a, b):
        a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
        return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
    out = {"set": name, "points": int(ref["P"]),
           "rel_err_out": rel(r["out"].cpu().numpy()[idx], ref["f"]),
           "rel_err_tan": rel(r["tan"].cpu().numpy()[idx], ref["g"]),
           "rel_err_loss": rel(r["loss"].cpu().numpy(), [float(ref["loss"])]),
           "rel_err_grad": rel(r["grad"].cpu().numpy(), ref["grad"])}
    c.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c5", choices=["c2", "c3", "c4", "c5"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="points of the CPU oracle sample (default: two chunks per core at 12 qubits)")
    ap.add_argument("--no-c1", action="store_true", help="skip the plain FP64 4-qubit wall-time leg")
    ap.add_argument("--no-total", action="store_true", help="skip the paper's total-loss leg")
    ap.add_argument("--no-training", action="store_true", help="skip the training-epoch leg")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-dense", action="store_true", help="skip the dense-block MFMA comparison leg")
    ap.add_argument("--no-paper-context", action="store_true",
                    help="skip the run of the paper's own circuit shape at its grid sizes")
    ap.add_argument("--tune", action="store_true", help="autotune the launch shape first")
    ap.add_argument("--no-separate", action="store_true",
                    help="skip timing the batched circuits as separate calls (uneven-batch workload only)")
    ap.add_argument("--no-graph", action="store_true",
                    help="time eager launches instead of replays of the step captured in a HIP graph")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 1 GiB device buffer three times (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": src.numel() * 4, "copy_bytes_written_per_launch": src.numel() * 4}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(sharding over several GPUs is designed but not built)"}))
        sys.exit(2)

    import numpy as np

    import workloads as W
    k = {"c2": 1, "c3": 2, "c4": 3, "c5": 4}[args.workload]
    cpu_line = None
    if k != 3 and not args.no_cpu_baseline:
        # the oracle's process pool forks, so it runs before this process initialises the GPU
        cpu_line = cpu_baseline(W.config(k), args.cpu_sample)
        log(f"bench: cpu {cpu_line}")

    import torch
    from paper_2506_23246_amd import _lib as L
    from paper_2506_23246_amd.api import Batch, Circuit, Context

    ctx = Context(0)
    dev = torch.device("cuda", 0)
    flags = L.QP_FLAG_TUNE if args.tune else 0

    if k == 3:
        ws_list = W.config(3)
        batch = Batch(ctx, [w.circuit for w in ws_list], [len(w.points) for w in ws_list])
        arr, bufs = batch.io([w.params for w in ws_list], [w.points for w in ws_list])
        P_total = sum(len(w.points) for w in ws_list)
        flops = sum(flops_per_point(w.circuit.n_params // 3, w.circuit.n) * len(w.points) for w in ws_list)
        flops_x = 0.0
        flops_mc = 0.0
        for w in ws_list:
            cq = Circuit(ctx, w.circuit)
            fx = executed_flops_per_point(cq.info(3), w.circuit.n, cq.info(12)) * len(w.points)
            flops_x += fx
            flops_mc += fx * matrix_core_share(cq.info(3), cq.info(12))
            cq.close()
        mc_share = flops_mc / flops_x if flops_x > 0 else 0.0

        def step():
            batch.run(arr, W.MaxwellDesc(W.LOSS_VACUUM), flags=0)
        if args.tune:
            batch.run(arr, W.MaxwellDesc(W.LOSS_VACUUM), flags=L.QP_FLAG_TUNE)
        cfg = {"workload": W.CONFIG_NAMES[3], "circuits": len(ws_list), "points_total": P_total,
               "work_items": batch.info(1), "work_items_3_to_8_qubits": batch.info(4),
               "grids_3_to_8_and_9_to_11_qubits": [batch.info(5), batch.info(6)]}
        w = None
    else:
        w = W.config(k)
        c = Circuit(ctx, w.circuit)
        P_total = len(w.points)
        prm = torch.tensor(w.params, device=dev)
        pts = torch.tensor(w.points, device=dev)
        bufs = {"out": torch.empty((P_total, 3), dtype=torch.float32, device=dev),
                "tan": torch.empty((P_total, 3, 3), dtype=torch.float32, device=dev),
                "loss": torch.empty(1, dtype=torch.float64, device=dev),
                "grad": torch.empty(w.circuit.n_params, dtype=torch.float32, device=dev)}
        F = c.info(3)
        flops = flops_per_point(F, w.circuit.n) * P_total
        flops_x = executed_flops_per_point(F, w.circuit.n, c.info(12)) * P_total
        mc_share = matrix_core_share(F, c.info(12))

        def step():
            c.maxwell(prm, pts, w.loss, bufs=bufs)
        if args.tune:
            c.maxwell(prm, pts, w.loss, bufs=bufs, flags=L.QP_FLAG_TUNE)
        cfg = {"workload": w.name, "n_qubits": w.circuit.n, "layers": w.circuit.n_params // (3 * w.circuit.n),
               "points": P_total, "params": w.circuit.n_params, "fused_gates": F, "rounds": c.info(4),
               "rounds_folded_into_encoding": c.info(11),
               "threads_per_wg": c.info(6), "points_per_tile": c.info(7), "lds_exchange_planes": c.info(8),
               "wg_per_cu": c.info(9), "loss": {0: "vacuum", 1: "dielectric split", 2: "dielectric intuitive"}[w.loss.kind]}

    log(f"bench: workload {cfg['workload']} P={P_total}; warmup {args.warmup}, steps {args.steps}")
    # The timed step is one replay of the whole sequence (gate table, fused kernel, FP64
    # reductions) captured in a HIP graph on a dedicated stream; --no-graph times eager launches.
    run_step, timing = step, "eager launches"
    gs = torch.cuda.Stream()
    ctx.use_stream(gs)
    with torch.cuda.stream(gs):
        step()                       # first use on this stream (launch attributes, plan upload)
    gs.synchronize()
    if not args.no_graph:
        try:
            if k == 3:
                def run_step():
                    batch.run(arr, W.MaxwellDesc(W.LOSS_VACUUM), graph=True)
            else:
                graph = torch.cuda.CUDAGraph()
                with torch.cuda.graph(graph, stream=gs):
                    step()
                run_step = graph.replay
            timing = "HIP graph replays"
        except Exception as e:  # pragma: no cover - reported, eager timing instead
            log(f"bench: graph capture failed ({e}); timing eager launches")
            run_step = step
    cfg["timing"] = timing
    with torch.cuda.stream(gs):
        for _ in range(args.warmup):
            run_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            run_step()
        torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1e3 / max(args.steps, 1)
    value = P_total / (ms_per_step / 1e3)
    log(f"bench: {ms_per_step:.3f} ms/step, {value:.4g} evals/s")

    # dominant kernel duration with HIP events on its own stream
    ctx.kernel_timing(True)
    kms = []
    with torch.cuda.stream(gs):
        for _ in range(max(3, min(args.steps, 10))):
            step()
            kms.append(ctx.last_kernel_ms())
    torch.cuda.synchronize()
    ctx.use_stream(torch.cuda.current_stream(dev))   # the extra legs below run on torch's stream
    ctx.kernel_timing(False)
    kms_avg = float(np.mean(kms))
    # the roofline's work is the arithmetic the kernel's algorithm needs (executed-flop count:
    # mul = 1, fma = 2, three-component gate statistic, opening stage folded); the larger
    # 256-flop-per-amplitude model of a gate-by-gate 2x2 product is reported beside it
    achieved = flops_x / (kms_avg / 1e3) / 1e12
    kname = "k_fused" if k != 3 else "k_batch"
    traffic, traffic_src = recorded_traffic(kname, cfg["workload"])
    # FP32 compute-bound: most of the arithmetic runs on the matrix cores (the gate products), the
    # rest (gate statistics) on the vector ALU; both units' FP32 peak is 157.3 TFLOP/s
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": traffic,
                "kernel": kname, "kernel_ms": round(kms_avg, 4),
                "algorithmic_flops_per_launch": flops_x, "matrix_core_flop_share": round(mc_share, 3),
                "model_256_flops_per_amp_gate_tflops": round(flops / (kms_avg / 1e3) / 1e12, 3)}
    if traffic_src:
        roofline["traffic_record"] = traffic_src
    log(f"bench: main kernel {kms_avg:.3f} ms, {achieved:.2f} TFLOP/s algorithmic")

    line = {"metric": "collocation-point circuit evals/s (fwd+3 input tangents+adjoint grad)", "value": round(value, 1),
            "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic", "config": cfg, "roofline": roofline}

    if w is not None and not args.no_parity:
        from oracle import qpinn_oracle as O
        idx = np.linspace(0, P_total - 1, 8).astype(int)
        f, g = O.simulate(w.circuit, w.params, w.points[idx])
        out = bufs["out"][idx].cpu().numpy()
        tan = bufs["tan"][idx].cpu().numpy()
        rel = lambda a, b: float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
        line["parity"] = {"timed_run_sampled_points": len(idx), "rel_err_out": rel(out, f), "rel_err_tan": rel(tan, g),
                          "loss": float(bufs["loss"].cpu()[0]), "grad_norm": float(bufs["grad"].norm().cpu())}
        stored = {4: "c5_first4096", 2: "c3_first16384"}.get(k)
        if stored:
            line["parity"]["stored_oracle_subsample"] = parity_vs_stored_oracle(ctx, w, stored)
        log(f"bench: parity {line['parity']}")

    if w is not None and not args.no_plain:
        P_sub = min(P_total, 4096 if w.circuit.n >= 12 else 16384)
        sub = torch.tensor(w.points[:P_sub], device=dev)
        c.plain_eval(prm, sub, precision=32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.plain_eval(prm, sub, precision=32)
        torch.cuda.synchronize()
        t_eval = time.perf_counter() - t0
        t0 = time.perf_counter()
        c.plain_maxwell_fd(prm, sub, w.loss, precision=32, k_begin=0, k_end=2)
        torch.cuda.synchronize()
        t_fd2 = time.perf_counter() - t0
        t_param = max(t_fd2 - t_eval, 0.0) / 2.0
        K = w.circuit.n_params
        t_full = (P_total / P_sub) * (t_eval + K * t_param)
        line["plain_gpu"] = {
            "what": "per-gate kernels on HBM state, FP32, tangents by central FD (7 forwards), parameter gradient "
                    "by central FD of the loss (2 FD-tangent evaluations per parameter)",
            "timed": f"{P_sub} points; 2 of {K} parameters; scaled linearly to {P_total} points and {K} parameters",
            "fwd_fd_tangents_evals_per_s": round(P_sub / t_eval, 1),
            "full_step_s_extrapolated": round(t_full, 3),
            "speedup_fused_vs_plain": round(t_full / (ms_per_step / 1e3), 1),
            "speedup_fused_vs_plain_fwd_tangents_only": round((P_total / P_sub) * t_eval / (ms_per_step / 1e3), 2)}
        log(f"bench: plain {line['plain_gpu']}")

    if w is not None and not args.no_dense and w.circuit.n >= 5:
        # dense 2^5 blocks on FP32 MFMA (streamed through HBM), same step on a point subset
        P_d = min(P_total, 16384)
        sub = torch.tensor(w.points[:P_d], device=dev)
        bd = {"out": torch.empty((P_d, 3), dtype=torch.float32, device=dev),
              "tan": torch.empty((P_d, 3, 3), dtype=torch.float32, device=dev),
              "loss": torch.empty(1, dtype=torch.float64, device=dev),
              "grad": torch.empty(w.circuit.n_params, dtype=torch.float32, device=dev)}
        c.maxwell(prm, sub, w.loss, bufs=bd, flags=L.QP_FLAG_DENSE_MFMA)
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            c.maxwell(prm, sub, w.loss, bufs=bd, flags=L.QP_FLAG_DENSE_MFMA)
        torch.cuda.synchronize()
        t_d = (time.perf_counter() - t0) / reps
        G = int(c.info(10))
        cols = 2 ** (w.circuit.n - 5)
        mm = 2.0 * 64 * 64 * cols                       # one 64x64 real block on one statevector
        flops_d = G * (12 * mm + 4 * 4 * 2 * 32 * 32 * cols) * P_d
        bytes_d = G * (12 * 2 + 8) * (2 ** w.circuit.n) * 8 * P_d
        line["dense_mfma"] = {
            "what": "the same fused Maxwell step with every gate run grouped into 32x32 complex blocks on "
                    "v_mfma_f32_32x32x2f32, statevectors streamed through HBM (amplitude-major)",
            "points": P_d, "blocks": G, "evals_per_s": round(P_d / t_d, 1),
            "relative_to_fused": round((P_d / t_d) / value, 4),
            "algorithmic_mfma_tflops": round(flops_d / t_d / 1e12, 2),
            "modelled_hbm_gbs": round(bytes_d / t_d / 1e9, 1)}
        log(f"bench: dense {line['dense_mfma']}")

    if k == 3 and not args.no_separate:
        # The same circuits, each run as its own fused Maxwell call (own plan, own launches and
        # reductions) back to back on one stream: what the one-launch uneven batch replaces.
        sep = []
        for wi in ws_list:
            ci = Circuit(ctx, wi.circuit)
            pi = torch.tensor(wi.params, device=dev)
            xi = torch.tensor(wi.points, device=dev)
            bi = {"out": torch.empty((len(wi.points), 3), dtype=torch.float32, device=dev),
                  "tan": torch.empty((len(wi.points), 3, 3), dtype=torch.float32, device=dev),
                  "loss": torch.empty(1, dtype=torch.float64, device=dev),
                  "grad": torch.empty(wi.circuit.n_params, dtype=torch.float32, device=dev)}
            sep.append((ci, pi, xi, bi))
        vac = W.MaxwellDesc(W.LOSS_VACUUM)

        def run_separate():
            for ci, pi, xi, bi in sep:
                ci.maxwell(pi, xi, vac, bufs=bi)
        run_separate()
        torch.cuda.synchronize()
        reps = max(3, min(args.steps, 10))
        t0 = time.perf_counter()
        for _ in range(reps):
            run_separate()
        torch.cuda.synchronize()
        t_sep = (time.perf_counter() - t0) / reps
        line["separate_launches"] = {
            "what": f"the same {len(sep)} circuits and points, one fused Maxwell call per circuit, "
                    "eager, back to back on one stream",
            "ms_per_step": round(t_sep * 1e3, 4), "evals_per_s": round(P_total / t_sep, 1),
            "batch_speedup": round(t_sep / (ms_per_step / 1e3), 3)}
        log(f"bench: separate {line['separate_launches']}")
        for ci, _, _, _ in sep:
            ci.close()
        del sep

    if w is not None and not args.no_paper_context and k == 4:
        # The paper's PQC shape (7 qubits, 4 layers of Rot + CNOT ring, RX(acos a) embedding of 7
        # angles produced by its classical layer) at the grid sizes of its timing table.  Angles and
        # their Jacobian are synthetic; context only, not a like-for-like comparison.
        pc = W.paper_context_circuit("basic")
        cc = Circuit(ctx, pc)
        rng = np.random.default_rng(7)
        prm_c = torch.tensor(rng.uniform(0, 2 * math.pi, pc.n_params).astype(np.float32), device=dev)
        ours = {}
        for side in (40, 87):
            Pc = side ** 3
            ang = torch.tensor(rng.uniform(0.0, math.pi, (Pc, pc.n)).astype(np.float32), device=dev)
            jac = torch.tensor(rng.standard_normal((Pc, pc.n, 3)).astype(np.float32), device=dev)
            cc.maxwell(prm_c, None, W.MaxwellDesc(), angles=ang, jac=jac)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(5):
                cc.maxwell(prm_c, None, W.MaxwellDesc(), angles=ang, jac=jac)
            torch.cuda.synchronize()
            ours[f"{side}^3"] = round(Pc / ((time.perf_counter() - t0) / 5), 1)
            del ang, jac
        # the paper's other ansatz families at the 40^3 grid (angle gradients included, as the hybrid model needs)
        per_ansatz = {}
        Pc = 40 ** 3
        ang = torch.tensor(rng.uniform(0.0, math.pi, (Pc, 7)).astype(np.float32), device=dev)
        jac = torch.tensor(rng.standard_normal((Pc, 7, 3)).astype(np.float32), device=dev)
        for name in ("basic", "strong", "noent", "cross_mesh", "cross_mesh_2rot", "cross_mesh_cnot"):
            pa = W.paper_context_circuit(name)
            ca = Circuit(ctx, pa)
            pr = torch.tensor(rng.uniform(0, 2 * math.pi, pa.n_params).astype(np.float32), device=dev)
            ca.maxwell(pr, None, W.MaxwellDesc(), angles=ang, jac=jac, input_grads=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(5):
                ca.maxwell(pr, None, W.MaxwellDesc(), angles=ang, jac=jac, input_grads=True)
            torch.cuda.synchronize()
            per_ansatz[name] = {"quantum_params": pa.n_params,
                                "evals_per_s": round(Pc / ((time.perf_counter() - t0) / 5), 1)}
            ca.close()
        del ang, jac
        line["paper_context"] = {
            "what": "the paper's circuit shape: 7 qubits x 4 layers, Rot + CNOT ring, RX(acos) embedding of given "
                    "angles, fused forward + 3 input tangents + Maxwell loss + adjoint gradient",
            "ours_evals_per_s": ours,
            "ansatz_families_40cubed_with_angle_gradients": per_ansatz,
            "paper_torq_points_per_s": {"40^3": 4.41e5, "87^3": 7.75e5},
            "paper_scope": "grid^3 / seconds per training epoch of the whole hybrid model (66848-parameter MLP, "
                           "the PQC, autograd input derivatives, all loss terms, backward, Adam) on NVIDIA L40S or "
                           "A100, precision not stated; context only"}
        log(f"bench: paper context {line['paper_context']['ours_evals_per_s']}")

    if w is not None and not args.no_total:
        # The paper's total loss (residuals + 10 IC + 10 symmetry + 10 energy) on the same points and a
        # 4096-point initial-condition plane: forward over [X; mirror images; IC plane], seeds, adjoint.
        xy = W.ic_plane_points(np.random.default_rng(77), 4096)
        tdesc = W.TotalLossDesc(phys=w.loss)
        c.total_loss(prm, pts, xy, tdesc)
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            r_tot = c.total_loss(prm, pts, xy, tdesc)
        torch.cuda.synchronize()
        t_tot = (time.perf_counter() - t0) / reps
        terms = r_tot["terms"].cpu().numpy()
        n_sets = 3 if w.loss.kind == W.LOSS_VACUUM else 2
        line["total_loss"] = {
            "what": "L_phys + 10 L_IC + 10 L_sym + 10 L_energy: packed forward (no tangents) over the "
                    f"{n_sets - 1} mirror image set(s) of the collocation points and a 4096-point IC plane, "
                    "one fused pass over the collocation points (forward with tangents, residual, energy and "
                    "symmetry seeds in the kernel, adjoint), the four terms, packed adjoint of the images",
            "points": P_total, "ic_points": 4096, "ms_per_step": round(t_tot * 1e3, 3),
            "collocation_evals_per_s": round(P_total / t_tot, 1),
            "relative_to_residual_only_step": round(t_tot / (ms_per_step / 1e3), 3),
            "terms": {"total": float(terms[0]), "phys": float(terms[1]), "ic": float(terms[2]),
                      "sym": float(terms[3]), "energy": float(terms[4])}}
        log(f"bench: total loss {line['total_loss']}")

    if k == 4 and not args.no_training:
        # Training epochs of the paper's hybrid model (classical network, 7-qubit 4-layer Basic
        # Entangling Layers, linear head) with the total loss and Adam, full batch, at the grid sizes of
        # the paper's runtime table; the same epoch for the circuit alone (qp_total_loss) at 40^3.
        from paper_2506_23246_amd.hybrid import HybridQPINN
        from paper_2506_23246_amd.train import grid_points, ic_plane, train_circuit, train_hybrid
        tr = {}
        for side in (40, 87):
            model = HybridQPINN(W.paper_context_circuit("basic"), ctx=ctx, seed=0).cuda()
            lg = train_hybrid(model, grid_points(side, device=dev), ic_plane(side, device=dev), W.TotalLossDesc(),
                              epochs=4)
            tr[f"{side}^3"] = {"s_per_epoch": round(lg.s_per_epoch(), 4), "loss_first_last": [lg.loss[0], lg.loss[-1]]}
            del model
        pc = W.paper_context_circuit("basic")
        pc.enc = W.Encoding()          # the circuit alone: cycled RY(pi c) encoding of the points
        cc = Circuit(ctx, pc)
        rng_t = np.random.default_rng(5)
        lg = train_circuit(cc, rng_t.uniform(0, 2 * math.pi, pc.n_params), grid_points(40, device=dev),
                           ic_plane(40, device=dev), W.TotalLossDesc(), epochs=4)
        line["training_epoch"] = {
            "what": "Adam epochs, full batch, total loss (residuals + 10 IC + 10 symmetry + 10 energy), paper's 7-qubit "
                    "4-layer circuit: hybrid = RFF + 256/128 tanh network + circuit (autograd Jacobian of the angles, "
                    "engine tangents and adjoint) + Linear(7, 3); circuit_alone = qp_total_loss on the circuit",
            "hybrid": tr, "circuit_alone_40^3_s_per_epoch": round(lg.s_per_epoch(), 4),
            "paper_torq_s_per_epoch": {"40^3": 0.145136, "87^3": 0.849967},
            "paper_scope": "TorQ, NVIDIA L40S or A100, precision not stated; the paper's model also has the periodic "
                           "input map; context only"}
        log(f"bench: training {line['training_epoch']}")

    if k == 4 and not args.no_c1:
        line["c1_plain_fp64"] = c1_plain_fp64(ctx, dev)
        log(f"bench: c1 {line['c1_plain_fp64']}")

    if cpu_line is not None:
        line["cpu_baseline"] = cpu_line

    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
