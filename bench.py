"""Benchmark: two-qubit-gate MPO updates per second at bond dimension 1024.

A step is one noisy two-qubit gate update (centre move + contraction + 16x16
channel + truncated SVD + entropy) on a saturated bulk bond,
chi_L = chi_M = chi_R = 1024, theta' of size 4096 x 4096.  The state is an
in-situ one from the precision workload: a 64-qubit chain evolved from
|0..0> by a depth-12 brickwork of Haar gates, each followed by two-qubit
depolarizing noise p = 0.01 (seed 0, chi_max = 1024, cutoff 1e-12; built in
FP32 mode, the fastest, and exported), where every bond of sites 4..59 sits at
chi = 1024.  Timed gates continue the brickwork on the bulk sites 16..46 with
fresh Haar gates (seed 1): one time step puts 16 gates on 16, 18, .., 46, the
next 15 on 17, .., 45, and the centre moves the brickwork needs (one per gate
within a step, back across the bulk between steps) are part of every step.
Inputs are resident in HBM before timing.

The FP32-MFMA path is the headline `value`; the FP64 path on the same gates
and snapshot is reported beside it, with the entropy error between the two
and against the CPU oracle on the first timed gate.  `roofline` is for the
kernel class with the largest event-measured time in the FP32 timed region,
`roofline_per_gate` for the whole gate against its nominal work;
`cpu_baseline` times the oracle on one bulk gate of the same snapshot.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--chi 1024]
                       [--no-cpu-baseline] [--cpu-single-thread]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "2q-gate MPO updates/sec at chi=1024 (FP32-MFMA vs FP64) + entropy err vs oracle"
HBM_PEAK = 8.0e12                              # bytes/s
PEAK = {"fp64": 78.6e12, "fp32": 157.3e12,   # dense MFMA (= vector) peaks of MI355X
        "bf16x3": 2.5e15}                      # BF16 dense MFMA peak


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def bulk_schedule(lo, hi, count, start_parity=1):
    """Sites of `count` gates of a brickwork restricted to sites lo..hi."""
    out, t = [], start_parity
    while len(out) < count:
        first = lo if (t % 2) == (lo % 2) else lo + 1
        for s in range(first, hi + 1, 2):
            if len(out) < count:
                out.append(s)
        t += 1
    return out


def build_snapshot(pm, mi, n, depth, p, chi, seed, prec="fp64"):
    draws = mi.ginibre_draws(n, depth, seed=seed)
    sup = pm.build_superops(draws, p, "pauli")
    st = pm.Mpo(n, chi, prec, "pauli")
    t0 = time.time()
    st.run_brickwork(depth, sup, chi, 1e-12, record=None)
    dims, centre = st.bond_dims()
    snap = st.export()
    st.close()
    return snap, dims, time.time() - t0


def timed_run(pm, torch, snap, n, chi, prec, sites, sups, warmup, steps, profile):
    """Warmup gates, then `steps` timed gates from the same snapshot.  With
    `profile`, every kernel launch is bracketed by HIP events on the engine's
    stream (per-launch durations and algorithmic work for the roofline); the
    events cost about a quarter of the run, so `value` comes from a pass
    without them and the roofline from a second pass over the same gates."""
    st = pm.Mpo(n, chi, prec, "pauli")
    st.import_state(snap)
    ent = []
    for g in range(warmup):
        ent.append(st.apply(sites[g], sups[g], chi, 1e-12).entropy)
    torch.cuda.synchronize()
    st.profile(profile)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g in range(warmup, warmup + steps):
        ent.append(st.apply(sites[g], sups[g], chi, 1e-12).entropy)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = st.profile_read() if profile else None
    dims = st.bond_dims()[0]
    st.close()
    return dt, np.array(ent), prof, dims


def roofline(prof, prec):
    """Roofline object for the kernel class with the largest measured time.
    The bound is the one its algorithmic intensity (flops per HBM byte) puts
    it under: MFMA above the precision's ridge point, HBM below it; the pair
    eigen-solver is FP64 vector-ALU work in every mode."""
    ks = prof["kernels"]
    name, k = max(ks.items(), key=lambda kv: kv[1]["ms"])
    t = k["ms"] * 1e-3
    launches = max(1, k["launches"])
    intensity = k["flops"] / k["bytes"] if k["bytes"] > 0 else float("inf")
    if name == "jacobi_eig64":
        bound, peak, ach, unit, scale = "alu", PEAK["fp64"], k["flops"] / t, "TFLOP/s", 1e12
    elif intensity < PEAK[prec] / HBM_PEAK:
        bound, peak, ach, unit, scale = "hbm", HBM_PEAK, k["bytes"] / t, "GB/s", 1e9
    else:
        bound, peak, ach, unit, scale = "mfma", PEAK[prec], k["flops"] / t, "TFLOP/s", 1e12
    return name, {"bound": bound, "achieved": ach / scale, "peak": peak / scale, "unit": unit,
                  "frac": ach / peak, "traffic": measured_traffic(name, prec), "kernel": name,
                  "launches": k["launches"], "avg_us": 1e3 * k["ms"] / launches,
                  "flops_per_launch": k["flops"] / launches,
                  "algorithmic_bytes_per_launch": k["bytes"] / launches,
                  "intensity_flop_per_byte": intensity,
                  "share_of_timed_region": k["ms"] / sum(v["ms"] for v in ks.values()),
                  "measured_in": "second pass over the same gates with per-launch HIP events"}


def nominal_gate_work(chi, prec):
    """Nominal real flops of one bulk gate at bond dimension chi (N = 4 chi, k = chi
    kept), split by the unit that bounds each phase, and the roofline time:
      theta 128 chi^3 + channel 2048 chi^2 + Gram 4 N^3 (Hermitian half)
      + right factor 8 k N^2 + centre move (QR + R A) 91 chi^3   -> contractions
      + eigen core (16/3) N^3 + 8 N^2 k (tridiagonalisation + back-transform) -> FP64
    Contractions run at the mode's MFMA peak (BF16x3: three BF16 products), the
    eigen core at the FP64 peak in every mode.  The fused lower bound on bytes
    reads and writes the two site tensors once: 16 chi^2 complex values."""
    N, k = 4 * chi, chi
    contr = 128.0 * chi ** 3 + 2048.0 * chi ** 2 + 4.0 * N ** 3 + 8.0 * k * N ** 2 + 91.0 * chi ** 3
    eig = (16.0 / 3.0) * N ** 3 + 8.0 * N ** 2 * k
    cpeak = {"fp64": PEAK["fp64"], "fp32": PEAK["fp32"], "bf16x3": PEAK["bf16x3"] / 3.0}[prec]
    csz = 16 if prec == "fp64" else 8
    t_roof = contr / cpeak + eig / PEAK["fp64"]
    return {"nominal_flops": contr + eig, "contraction_flops": contr, "eigen_core_flops": eig,
            "t_roof_ms": 1e3 * t_roof, "fused_min_bytes": 16.0 * chi * chi * csz}


def per_gate_roofline(prof, prec, chi, ms_per_gate, gates):
    """Whole-gate roofline: nominal work / measured time, plus the algorithmic bytes
    the kernels of one gate actually move (all launches) against the fused bound."""
    w = nominal_gate_work(chi, prec)
    ks = prof["kernels"]
    alg_bytes = sum(v["bytes"] for v in ks.values()) / max(1, gates)
    alg_flops = sum(v["flops"] for v in ks.values()) / max(1, gates)
    return {"t_roof_ms": w["t_roof_ms"], "ms_per_gate": ms_per_gate, "frac": w["t_roof_ms"] / ms_per_gate,
            "nominal_flops_per_gate": w["nominal_flops"],
            "counted_flops_per_gate": alg_flops, "flops_ratio_counted_to_nominal": alg_flops / w["nominal_flops"],
            "algorithmic_bytes_per_gate": alg_bytes, "fused_min_bytes_per_gate": w["fused_min_bytes"],
            "bytes_ratio_to_fused_min": alg_bytes / w["fused_min_bytes"]}


def source_digest(spec):
    """sha256 over named pieces of source files, spec = {relative path: [names]}:
    a function is taken from its name at its definition (the name followed by
    its parameter list and an opening brace) through its closing brace, a
    constant from `constexpr int NAME =` through the semicolon.  None if a file
    or a name is missing."""
    import hashlib
    import re
    h = hashlib.sha256()
    for rel in sorted(spec):
        try:
            text = open(os.path.join(ROOT, rel)).read()
        except OSError:
            return None
        for name in spec[rel]:
            piece = None
            m = re.search(r"constexpr\s+int\s+" + re.escape(name) + r"\s*=[^;]*;", text)
            if m:
                piece = m.group(0)
            for m in re.finditer(r"\b" + re.escape(name) + r"\s*\(", text):
                if piece is not None:
                    break
                i, depth = m.end() - 1, 0
                while i < len(text):           # the parameter list
                    depth += {"(": 1, ")": -1}.get(text[i], 0)
                    i += 1
                    if depth == 0:
                        break
                k = i
                while k < len(text) and text[k] in " \t\n":
                    k += 1
                if k >= len(text) or text[k] != "{":
                    continue                    # a call or a declaration
                depth = 0
                while k < len(text):           # the body
                    depth += {"{": 1, "}": -1}.get(text[k], 0)
                    k += 1
                    if depth == 0:
                        break
                piece = text[m.start():k]
            if piece is None:
                return None
            h.update(rel.encode() + b"\0" + name.encode() + b"\0" + piece.encode() + b"\0")
    return h.hexdigest()


def measured_traffic(kernel, prec):
    """HBM bytes per launch from the committed rocprofv3 counter runs, or None
    when the kernel's source changed since they were taken: the record names
    either whole files (sha256 of each) or the kernel's own functions and
    constants (one digest over them, `source_digest`)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    for rel, sha in rec.get("source_sha256", {}).items():
        try:
            if hashlib.sha256(open(os.path.join(ROOT, rel), "rb").read()).hexdigest() != sha:
                return None
        except OSError:
            return None
    dig = rec.get("source_digest")
    if dig is not None and source_digest(dig.get("spec", {})) != dig.get("sha256"):
        return None
    if rec.get("precision") != prec or kernel not in rec.get("kernels", {}):
        return None
    return rec["kernels"][kernel]["bytes_per_launch"]


def batch_measurement(pm, mi, torch, count, depth_cap=4, chi_cap=64, streams=16):
    """The batched workload's 128 circuits (circuit i: n even in 16..96, depth in
    [n/2, n], p in [0.005, 0.03], chi_max in {64..512}, all from PCG64(i)) with
    depth and chi_max capped so that the run stays short: aggregate updates/s
    on one stream (the circuits one after the other), on `streams` concurrent
    streams, and on `streams` streams with the Jacobi sweeps replayed from
    captured HIP graphs; the three must agree bit for bit."""
    circuits, sups, ngates = [], [], 0
    for i in range(count):
        spec, draws = mi.batch_circuit(i)
        depth, chi = min(spec.depth, depth_cap), min(spec.chi_max, chi_cap)
        g = pm.n_schedule_gates(spec.n, depth)
        circuits.append((spec.n, depth, chi, 1e-12))
        sups.append(pm.build_superops(draws[:g], spec.p, "pauli"))
        ngates += g
    res = {}
    outs = {}
    for label, ns, graphs in (("sequential", 1, False), (f"streams{streams}", streams, False),
                              (f"streams{streams}_graphs", streams, True)):
        log(f"batch: {count} circuits, {ngates} gates, {ns} stream(s), graphs {graphs}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs[label] = pm.batch_run(circuits, sups, "fp32", "pauli", n_streams=ns, use_graph=graphs)
        dt = time.perf_counter() - t0
        res[label] = ngates / dt
    ref = outs["sequential"]
    same = all(np.array_equal(a["S"], b["S"]) and np.array_equal(a["Z"], b["Z"])
               for o in outs.values() for a, b in zip(ref, o))
    return {"workload": f"{count} circuits of the batched workload (seeds 0..{count - 1}), depth<={depth_cap}, "
                        f"chi_max<={chi_cap}, FP32-MFMA", "gates": ngates,
            **{f"{k}_updates_per_s": v for k, v in res.items()},
            "speedup_streams": res[f"streams{streams}"] / res["sequential"],
            "speedup_streams_graphs": res[f"streams{streams}_graphs"] / res["sequential"],
            "results_identical": bool(same)}


def adjoint_measurement(pm, mi, torch, n=32, depth=24, p=0.01, chi=256):
    """Frozen-projector gradient of O = sum_i Tr[Z_i rho_D] for n = 32, depth 24,
    p = 0.01, chi_max = 256 (seed 0): forward and backward times, the Euler
    identity sum M_g dO/dM_g = O over every gate, and dO/dp by the chain rule
    through M_g = diag(1, 1-16p/15, ...) S_U in the Pauli basis."""
    draws = mi.ginibre_draws(n, depth, seed=0)
    sup = pm.build_superops(draws, p, "pauli")
    log(f"adjoint: n={n} depth={depth} p={p} chi={chi} ({len(sup)} gates)")
    st = pm.Mpo(n, chi, "fp64", "pauli")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.run_brickwork(depth, sup, chi, 1e-12, record=None)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    st.close()
    st = pm.Mpo(n, chi, "fp64", "pauli")
    t0 = time.perf_counter()
    O, grads, comax = st.adjoint_brickwork(depth, sup, chi, 1e-12, checkpoint_every=4)
    t_adj = time.perf_counter() - t0
    st.close()
    euler = np.einsum("gij,gij->g", sup, grads)
    su = pm.build_superops(draws, 0.0, "pauli")
    dmdp = np.concatenate([[0.0], np.full(15, -16.0 / 15.0)])[None, :, None] * su
    dO_dp = float(np.einsum("gij,gij->", grads, dmdp).real)
    return {"workload": f"n={n}, depth {depth}, p={p}, chi_max={chi}, seed 0, FP64, O = sum_i Tr[Z_i rho_D], "
                        f"checkpoints every 4 time steps (segment recompute)",
            "gates": int(len(sup)), "forward_seconds": t_fwd, "forward_plus_adjoint_seconds": t_adj,
            "backward_seconds": t_adj - t_fwd, "O": O, "dO_dp": dO_dp,
            "euler_max_rel_dev": float(np.abs(euler - O).max() / abs(O)), "costate_max_bond": comax}


def cpu_baseline(snap_bytes, pm, site, sup, chi, threads=None):
    """Oracle (numpy complex128) on one bulk gate of the same snapshot: the
    centre is first moved next to the gate from the side the GPU comes from
    (untimed), then the gate is timed with the one QR move it needs, the
    contraction, the map and the gesdd split.  Both sides then move the centre
    through the same bonds, which matters for the comparison: the snapshot is
    canonical only to the precision it was built in, so a detour across other
    bonds would change the local split at that level.
    threads: BLAS threads (None = all)."""
    from oracle import mpo as omp
    from threadpoolctl import threadpool_info, threadpool_limits
    n, basis, centre, tensors = pm.snapshot_to_tensors(snap_bytes)
    m = omp.MPO.__new__(omp.MPO)
    m.n, m.basis, m.A, m.centre = n, "pauli", tensors, centre
    target = site + 1 if centre > site else max(0, site - 1)
    t0 = time.perf_counter()
    while m.centre != target:      # untimed: bring the centre next to the gate
        m.move_centre(m.centre + (1 if m.centre < target else -1))
        if abs(m.centre - target) % 8 == 0:
            log(f"  oracle centre at {m.centre} ({time.perf_counter() - t0:.0f} s)")
    log(f"  oracle gate at site {site}")
    with threadpool_limits(limits=threads, user_api="blas"):
        cores = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] + [1])
        t0 = time.perf_counter()
        info = m.apply_gate(site, sup, chi, 1e-12)
        dt = time.perf_counter() - t0
    return dt, info, cores


def host_description():
    """CPU model, logical CPUs and BLAS library of the host the oracle ran on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = None
    try:
        from threadpoolctl import threadpool_info
        libs = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        if libs:
            blas = f"{libs[0].get('internal_api')} {libs[0].get('version')}"
    except Exception:
        pass
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "blas": blas,
            "numpy": np.__version__}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--chi", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-single-thread", action="store_true",
                    help="also time the oracle gate with one BLAS thread (several minutes)")
    ap.add_argument("--precisions", default="fp32,fp64,bf16x3")
    ap.add_argument("--save-snapshot", default=None, help="write the in-situ snapshot to this file")
    ap.add_argument("--load-snapshot", default=None, help="reuse a snapshot written by --save-snapshot")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--batch-circuits", type=int, default=128)
    ap.add_argument("--copy-probe", action="store_true",
                    help="copy a 256 MiB device buffer 4 times first (traffic-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import mpo_inputs as mi
    import paper_2003_13163_amd as pm
    pm.library()
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)

    if args.copy_probe:
        x = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(4):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    n, depth, p, chi, seed = 64, 12, 0.01, args.chi, 0
    if args.load_snapshot:
        snap = open(args.load_snapshot, "rb").read()
        dims = [int(v) for v in np.frombuffer(snap, dtype=np.int64, count=n - 1, offset=32)]
        log(f"loaded snapshot {args.load_snapshot}: bond dims {dims}")
    else:
        log(f"building in-situ snapshot: n={n} depth={depth} p={p} chi={chi}")
        snap, dims, t_warm = build_snapshot(pm, mi, n, depth, p, chi, seed, prec="fp32")
        log(f"  bond dims {dims} ({t_warm:.1f} s)")
        if args.save_snapshot:
            with open(args.save_snapshot, "wb") as f:
                f.write(snap)
    lo, hi = 16, 46
    total = args.warmup + args.steps
    # the next time step (depth + 1) puts gates on even sites when depth is even
    sites = bulk_schedule(lo, hi, total, start_parity=depth % 2)
    draws = mi.ginibre_draws(n, 2 * total + 4, seed=seed + 1)
    sups = pm.build_superops(draws[:total], p, "pauli")

    res = {}
    for prec in args.precisions.split(","):
        log(f"timing {prec}: warmup {args.warmup} + {args.steps} gates")
        dt, ent, _, dims_after = timed_run(pm, torch, snap, n, chi, prec, sites, sups,
                                           args.warmup, args.steps, False)
        log(f"  {prec}: {args.steps / dt:.3f} updates/s ({1e3 * dt / args.steps:.1f} ms/update)")
        dtp, entp, prof, _ = timed_run(pm, torch, snap, n, chi, prec, sites, sups,
                                       args.warmup, args.steps, True)
        log(f"  {prec} with per-launch events: {1e3 * dtp / args.steps:.1f} ms/update, svd {prof['svd']}")
        if not np.array_equal(ent, entp):
            raise SystemExit(f"{prec}: the profiled pass differs from the timed pass")
        res[prec] = {"seconds": dt, "seconds_profiled": dtp, "entropy": ent, "prof": prof,
                     "dims": dims_after}

    head = "fp32" if "fp32" in res else next(iter(res))
    value = args.steps / res[head]["seconds"]
    rl_name, rl = roofline(res[head]["prof"], head)
    out = {
        "metric": METRIC, "value": value, "unit": "updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * res[head]["seconds"] / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if head == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": f"bulk noisy 2q gate at chi={chi} (theta' {4 * chi}x{4 * chi}) on an "
                               f"in-situ {n}-qubit state (depth-{depth} Haar+depolarizing p={p} "
                               f"brickwork, seed {seed}, chi_max={chi}), brickwork gates on sites "
                               f"{lo}..{hi} with their centre moves",
                   "chi": chi, "n": n, "p": p, "cutoff": 1e-12, "basis": "pauli",
                   "bond_dims": dims},
        "roofline": rl,
        "roofline_per_gate": per_gate_roofline(res[head]["prof"], head, chi,
                                               1e3 * res[head]["seconds"] / args.steps, args.steps),
    }
    for other, dt_name in (("fp64", "f64"), ("bf16x3", "f32 storage, split-bf16x3 products")):
        if other in res and other != head:
            out[other] = {"value": args.steps / res[other]["seconds"],
                          "ms_per_step": 1e3 * res[other]["seconds"] / args.steps, "dtype": dt_name,
                          "roofline": roofline(res[other]["prof"], other)[1],
                          "roofline_per_gate": per_gate_roofline(res[other]["prof"], other, chi,
                                                                 1e3 * res[other]["seconds"] / args.steps,
                                                                 args.steps)}
    if "fp64" in res:
        err = out.setdefault("entropy_error", {})
        for prec in res:
            if prec != "fp64":
                err[f"{prec}_vs_fp64_max_abs"] = float(np.abs(res[prec]["entropy"] -
                                                              res["fp64"]["entropy"]).max())
    out["kernels"] = {k: {kk: vv for kk, vv in v["prof"]["kernels"].items() if vv["launches"]}
                      for k, v in res.items()}
    out["svd"] = {k: v["prof"]["svd"] for k, v in res.items()}

    if not args.no_batch:
        out["batch"] = batch_measurement(pm, mi, torch, args.batch_circuits)
        log("  " + json.dumps(out["batch"]))
    if not args.no_adjoint:
        out["adjoint"] = adjoint_measurement(pm, mi, torch)
        log("  " + json.dumps(out["adjoint"]))

    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on the first bulk gate of the snapshot")
        dt, info, cores = cpu_baseline(snap, pm, sites[0], sups[0], chi)
        out["cpu_baseline"] = {"value": 1.0 / dt, "unit": "updates/s", "cores": cores,
                               "kind": "oracle", "host": host_description(),
                               "sample": f"1 bulk gate (site {sites[0]}, chi={chi}, with its one QR "
                                         f"move) of the same snapshot, numpy complex128 gesdd, {dt:.1f} s"}
        if args.cpu_single_thread:
            log("cpu baseline: the same gate with one BLAS thread")
            dt1, _, c1 = cpu_baseline(snap, pm, sites[0], sups[0], chi, threads=1)
            out["cpu_baseline"]["single_thread"] = {"value": 1.0 / dt1, "unit": "updates/s", "cores": c1,
                                                    "seconds": dt1}
        err = out.setdefault("entropy_error", {})
        for prec in res:
            err[f"{prec}_vs_oracle_first_gate"] = abs(float(res[prec]["entropy"][0]) - info.entropy)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
