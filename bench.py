"""Throughput of the fused stream-and-collide step on one MI355X.

Headline workload: the lock exchange on 1024 x 64 x 128 nodes, D3Q27 cumulant
collision + D3Q7 scalar, Re_b = 30000, Smagorinsky C_s = 0.1, Sc_T = 1,
g' = 1e-4, FP32 storage and arithmetic (synthetic initial state: step
function in the concentration with seeded +-1e-3 noise at the gate). A step
is one launch of the fused kernel over every node. Also measured on the same
GPU: FP16 / BF16 storage of the same model on 2048 x 128 x 256 nodes, and
the D3Q19 BGK + Smagorinsky + D3Q6 model on the headline grid.

Timing: W warm-up steps, then K steps between HIP events recorded on the
stream the kernels run on (torch's current stream, handed to the library).
MNUPS = nodes * K / seconds / 1e6. Algorithmic HBM bytes per node update:
one read and one write of every population, 2 * Q * bytes (272 B for the
cumulant model in FP32). The oracle (FP64, CPU) is timed on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "cumulant27_q7_1024x64x128_fp32": dict(nx=1024, ny=64, nz=128, model=0, storage="f32"),
    # the closure as printed in Eq. 32 with the paper's C_s = 0.03 and Sc_T = C_s
    # (Sec. 2.3.1): the setting in which model 2 runs the whole lock exchange at
    # Re_b = 30000 (with C_s = 0.1 in the standard form and Sc_T = 1 its D3Q6
    # scalar goes unstable near t~ = 5.6)
    "bgk19_smag_q6_1024x64x128_fp32": dict(nx=1024, ny=64, nz=128, model=1, storage="f32", cs=0.03,
                                           sc_t=0.03, paper_form=True),
    "cumulant27_fcm27_1024x64x128_fp32": dict(nx=1024, ny=64, nz=128, model=2, storage="f32"),
    "cumulant27_fcm27_2048x128x256_fp16": dict(nx=2048, ny=128, nz=256, model=2, storage="f16"),
    # the parametrised cumulant with the third-order limiter and no LES (the
    # paper's VirtualFluids configuration)
    "cumulant27param_fcm27_1024x64x128_fp32": dict(nx=1024, ny=64, nz=128, model=2, storage="f32",
                                                   param=True),
    "cumulant27param_fcm27_2048x128x256_fp16": dict(nx=2048, ny=128, nz=256, model=2, storage="f16",
                                                    param=True),
    "cumulant27_q7_2048x128x256_fp32": dict(nx=2048, ny=128, nz=256, model=0, storage="f32"),
    "cumulant27_q7_2048x128x256_fp16": dict(nx=2048, ny=128, nz=256, model=0, storage="f16"),
    "cumulant27_q7_2048x128x256_bf16": dict(nx=2048, ny=128, nz=256, model=0, storage="bf16"),
    "cumulant27_q7_2048x128x256_bf16_f16s": dict(nx=2048, ny=128, nz=256, model=0, storage="bf16_f16s"),
    "cumulant27_q7_4096x256x512_fp16": dict(nx=4096, ny=256, nz=512, model=0, storage="f16"),
    "cumulant27_q7_4096x256x512_bf16": dict(nx=4096, ny=256, nz=512, model=0, storage="bf16"),
    "cumulant27_q7_4096x256x512_bf16_f16s": dict(nx=4096, ny=256, nz=512, model=0, storage="bf16_f16s"),
}
HEADLINE = "cumulant27_q7_1024x64x128_fp32"
VARIANTS = ["cumulant27_q7_2048x128x256_fp16", "cumulant27_q7_2048x128x256_bf16",
            "cumulant27_q7_2048x128x256_bf16_f16s", "cumulant27_q7_4096x256x512_fp16",
            "bgk19_smag_q6_1024x64x128_fp32", "cumulant27_fcm27_1024x64x128_fp32",
            "cumulant27_fcm27_2048x128x256_fp16", "cumulant27param_fcm27_1024x64x128_fp32",
            "cumulant27param_fcm27_2048x128x256_fp16"]


def measure_adjoint(nx=256, ny=16, nz=32, n_steps=2000, k_ckpt=100, model=0, param=False):
    """Differentiation form: one lbm_adjoint_run (forward with checkpoints,
    recompute, hand-written adjoint) of the lock exchange, FP32, Re_b = 1000,
    C_s = 0.1, Sc_T = 1 (param: the parametrised cumulant with limiter 1e-2
    and no LES, Re_b = 30000). MNUPS counts the n_steps node updates of the
    differentiated run; the algorithmic bytes are those of the passes made: a
    forward step (2 Q 4 B per node) per step, one per recomputed step, a
    reverse step (3 Q 4 B) per step and one initial copy, Q the populations
    per node. The workspace is allocated before the timed region, and one
    untimed run of the same size comes first (it loads the kernels and makes
    the run's second stream); the second run is timed with HIP events on the
    library's stream."""
    import torch

    import paper_2112_08479_amd as pkg
    if param:
        cfg = pkg.Config(nx, ny, nz, model=model, storage=pkg.F32, re_b=30000.0, parametrized=True,
                         limiter=1e-2)
    else:
        cfg = pkg.Config(nx, ny, nz, model=model, storage=pkg.F32, re_b=1000.0, cs_smag=0.1, sc_t=1.0)
    lat = pkg.Lattice(cfg)
    # workspace and gradient buffer allocated before the timed region
    ws = torch.empty(lat.adjoint_workspace_bytes(n_steps, k_ckpt), dtype=torch.uint8, device="cuda")
    gchi = torch.empty((nz, ny, nx), dtype=torch.float64, device="cuda")
    lat.init_lock_exchange(0.125, 1e-3, 0)
    lat.adjoint_run(n_steps, k_ckpt, ws=ws, gchi=gchi)  # warm-up
    lat.init_lock_exchange(0.125, 1e-3, 0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(lat.stream)
    J, dcs, dsct, g = lat.adjoint_run(n_steps, k_ckpt, ws=ws, gchi=gchi)
    e1.record(lat.stream)
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) * 1e-3
    del ws, gchi
    n = cfg.n
    q = lat.params["q_flow"] + lat.params["q_scalar"]
    lat.close()
    # the passes actually made: n forward steps, the recomputed steps of every
    # segment but the last (whose states the forward pass kept), n reverse
    # steps, and the copy of the initial state into the first checkpoint
    nseg = -(-n_steps // k_ckpt)
    recomputed = (nseg - 1) * (k_ckpt - 1)
    bpn = (n_steps * 2 * q * 4 + recomputed * 2 * q * 4 + n_steps * 3 * q * 4 + 2 * q * 4) / n_steps
    mnups = n * n_steps / dt / 1e6
    name = ["cumulant27_q7", "bgk19_smag_q6", "cumulant27_fcm27"][model]
    if param:
        name = name.replace("cumulant27", "cumulant27param")
    return {"workload": f"adjoint_{name}_{nx}x{ny}x{nz}_fp32_{n_steps}steps_k{k_ckpt}",
            "nodes": n, "steps": n_steps, "recomputed_steps": recomputed, "seconds": dt, "MNUPS": mnups,
            "bytes_per_node_update": bpn, "GB_per_s": mnups * 1e6 * bpn / 1e9,
            "J": J, "dJ_dcs": dcs, "dJ_dsct": dsct, "hbm_frac": mnups * 1e6 * bpn / 1e9 / HBM_PEAK_GBS,
            "note": ("state fits the 256 MB last-level cache and the run is bound by the kernels' "
                     "latency: not an HBM roofline case" if n * q * 4 < (256 << 20) else "HBM resident")}


# adjoint runs: the 256 x 16 x 32 workload (2000 steps, checkpoints every 100)
# and 100 steps of the benchmark grid (checkpoints every 25)
ADJOINT_RUNS = {
    "c3_cumulant27_q7": dict(),
    "cumulant27_q7_1024x64x128": dict(nx=1024, ny=64, nz=128, n_steps=100, k_ckpt=25),
    "cumulant27_fcm27_1024x64x128": dict(nx=1024, ny=64, nz=128, n_steps=100, k_ckpt=25, model=2),
    "cumulant27param_fcm27_1024x64x128": dict(nx=1024, ny=64, nz=128, n_steps=100, k_ckpt=25, model=2,
                                              param=True),
}


def precision_report(steps=2000):
    """FP16 / BF16 storage against FP32 storage on 2048 x 128 x 256 nodes
    (model 1, the benchmark physics): front position, L1 velocity difference
    and mass drift after `steps` steps."""
    import torch

    import paper_2112_08479_amd as pkg
    out, ref = {}, None
    for name, st in (("fp32", pkg.F32), ("fp16", pkg.F16), ("bf16", pkg.BF16), ("bf16_f16s", pkg.BF16_F16S)):
        cfg = pkg.Config(2048, 128, 256, model=0, storage=st, re_b=30000.0, cs_smag=0.1, sc_t=1.0)
        lat = pkg.Lattice(cfg)
        lat.init_lock_exchange(0.125, 1e-3, 0)
        lat.step(steps)
        d = lat.diagnostics(raise_unstable=False)
        m = lat.moments(pkg.OUT_F32)
        u = torch.stack([m["ux"], m["uy"], m["uz"]])
        del m
        row = {"x_f": d["x_f"], "x_f_nd": d["x_f_nd"], "mass_drift": (d["mass"] - d["mass0"]) / d["mass0"],
               "chi_mass_drift": (d["chi_mass"] - d["chi_mass0"]) / d["chi_mass0"],
               "nonfinite": d["nonfinite"]}
        if ref is None:
            ref = (u.clone(), d["x_f"])
        else:
            row["front_rel_diff_vs_fp32"] = abs(d["x_f"] - ref[1]) / abs(ref[1])
            row["l1_velocity_diff_vs_fp32"] = float((u - ref[0]).abs().sum() / ref[0].abs().sum())
        out[name] = row
        del u
        lat.close()
        torch.cuda.empty_cache()
    return {"precision_report": "2048x128x256 cumulant27_q7, Re_b 30000, C_s 0.1", "steps": steps, **out}


def kernel_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2112_08479_amd", "csrc")
    for n in ("lattice.h", "collide.h", "runtime.h", "kernels.hip"):
        with open(os.path.join(d, n), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measure(name, steps, warmup):
    import torch

    import paper_2112_08479_amd as pkg
    w = WORKLOADS[name]
    st = {"f64": pkg.F64, "f32": pkg.F32, "f16": pkg.F16, "bf16": pkg.BF16, "bf16_f16s": pkg.BF16_F16S}[w["storage"]]
    par = w.get("param", False)
    cfg = pkg.Config(w["nx"], w["ny"], w["nz"], model=w["model"], storage=st, re_b=30000.0,
                     g_prime=1e-4, cs_smag=0.0 if par else w.get("cs", 0.1), sc_t=w.get("sc_t", 1.0),
                     smag_paper_form=w.get("paper_form", False), parametrized=par,
                     limiter=1e-2 if par else 0.0)
    lat = pkg.Lattice(cfg)
    lat.init_lock_exchange(0.125, 1e-3, 0)
    lat.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(lat.stream)
    lat.step(steps)
    e1.record(lat.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    d = lat.diagnostics(raise_unstable=False)
    q = lat.params["q_flow"] + lat.params["q_scalar"]
    es = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2, "bf16_f16s": 2}[w["storage"]]
    bpn = 2 * q * es
    n = cfg.n
    lat.close()
    del lat
    torch.cuda.empty_cache()
    mnups = n * steps / (ms * 1e-3) / 1e6
    gbs = mnups * 1e6 * bpn / 1e9
    return {"workload": name, "nodes": n, "steps": steps, "ms_per_step": ms / steps,
            "MNUPS": mnups, "bytes_per_node_update": bpn, "GB_per_s": gbs,
            "hbm_frac": gbs / HBM_PEAK_GBS, "nonfinite": d["nonfinite"], "mass_drift":
            (d["mass"] - d["mass0"]) / d["mass0"], "x_f_nd": d["x_f_nd"]}


def stream_copy(nbytes=2 << 30, reps=10):
    """Device-to-device copy of nbytes with the library's plain streaming copy
    kernel: the achievable read+write bandwidth on this GPU, and a kernel of
    known size that scales the HBM byte counters of the profiles."""
    import torch

    import paper_2112_08479_amd as pkg
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    s_ = torch.cuda.current_stream()
    pkg.stream_copy(b, a, nbytes, s_)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s_)
    for _ in range(reps):
        pkg.stream_copy(b, a, nbytes, s_)
    e1.record(s_)
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) * 1e-3 / reps
    assert bool((b[:: 1 << 20] == 1.0).all())
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_per_copy": 2 * nbytes, "GB_per_s": 2 * nbytes / s / 1e9}


def traffic_for(name, bpn_launch):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    p = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        rec = json.load(fh).get(name)
    if not rec or rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(reps=3, steps_per_rep=2, warmup=1):
    """The FP64 oracle, as it stands, on a 1024 x 64 x 8 slab of the headline
    workload (its full x-y extent, 8 of its 128 z-layers, the same physical
    parameters and lock-exchange initial state): `warmup` untimed steps, then
    `reps` timed repetitions of `steps_per_rep` steps; the value is the median
    repetition's rate (about 10-20 s of CPU work in all)."""
    import statistics

    import torch

    from oracle import lbm as olbm
    from oracle.params import Config as OConfig
    from oracle.params import derive
    torch.set_num_threads(os.cpu_count() or 1)
    cores = torch.get_num_threads()
    full = OConfig(1024, 64, 128, model=0, re_b=30000.0, cs_smag=0.1)
    P = derive(full)
    slab = OConfig(1024, 64, 8, model=0, re_b=30000.0, cs_smag=0.1)
    f, phi = olbm.init_state(P, olbm.chi0_lock_exchange(slab, 0.125, 1e-3, 0))
    n = slab.nx * slab.ny * slab.nz
    for _ in range(warmup):
        f, phi = olbm.step(f, phi, P)
    rates = []
    for _ in range(reps):
        t0 = time.time()
        for _ in range(steps_per_rep):
            f, phi = olbm.step(f, phi, P)
        rates.append(n * steps_per_rep / (time.time() - t0) / 1e6)
    cpu = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    med = statistics.median(rates)
    return {"value": med, "unit": "MNUPS", "cores": cores, "kind": "oracle",
            "sample": f"FP64 oracle on a 1024x64x8 slab (z-layers of the 1024x64x128 workload, same "
                      f"parameters): {warmup} warm-up step, then the median of {reps} repetitions of "
                      f"{steps_per_rep} steps (MNUPS {', '.join(f'{r:.3f}' for r in rates)}) on "
                      f"{cores} threads of {cpu}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default=HEADLINE, choices=sorted(WORKLOADS))
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", action="store_true",
                    help="only the FP16/BF16 vs FP32 storage comparison on 2048x128x256")
    ap.add_argument("--adjoint", choices=sorted(ADJOINT_RUNS) + ["all"],
                    help="only the differentiation form: one adjoint run per JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("the library runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.precision:
        print(json.dumps(precision_report()), flush=True)
        return
    if args.adjoint:
        # the plain copy kernel runs first: it calibrates the HBM byte counters
        # of a profile taken of this command
        copy = stream_copy()
        print(json.dumps({"progress": "stream_copy", **copy}), file=sys.stderr, flush=True)
        for name in (sorted(ADJOINT_RUNS) if args.adjoint == "all" else [args.adjoint]):
            print(json.dumps(measure_adjoint(**ADJOINT_RUNS[name])), flush=True)
        return
    copy = stream_copy()
    print(json.dumps({"progress": "stream_copy", **copy}), file=sys.stderr, flush=True)
    head = measure(args.workload, args.steps, args.warmup)
    print(json.dumps({"progress": "headline", **head}), file=sys.stderr, flush=True)
    variants = []
    if not args.no_variants:
        for v in VARIANTS:
            if v == args.workload:
                continue
            r = measure(v, max(50, args.steps // 4), min(args.warmup, 50))
            print(json.dumps({"progress": "variant", **r}), file=sys.stderr, flush=True)
            variants.append(r)
        for name in sorted(ADJOINT_RUNS):
            r = measure_adjoint(**ADJOINT_RUNS[name])
            print(json.dumps({"progress": "adjoint", **r}), file=sys.stderr, flush=True)
            variants.append(r)
    cpu = None if args.no_cpu_baseline else cpu_baseline()
    launch_bytes = head["bytes_per_node_update"] * head["nodes"]
    achieved = launch_bytes / (head["ms_per_step"] * 1e-3) / 1e9
    w = WORKLOADS[args.workload]
    line = {
        "metric": "MNUPS (node updates per second / 1e6) of the fused stream-and-collide step",
        "value": head["MNUPS"],
        "unit": "MNUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f16": "f16-storage/f32", "bf16": "bf16-storage/f32",
                  "bf16_f16s": "bf16-flow/f16-scalar-storage/f32", "f64": "f64"}[w["storage"]],
        "data": "synthetic",
        "config": {"workload": args.workload, "nx": w["nx"], "ny": w["ny"], "nz": w["nz"],
                   "model": ["cumulant27_q7", "bgk19_smag_q6", "cumulant27_fcm27"][w["model"]], "re_b": 30000.0,
                   "cs_smag": 0.0 if w.get("param") else 0.1, "sc_t": 1.0, "g_prime": 1e-4,
                   "cumulant_rates": "parametrised, limiter 1e-2" if w.get("param") else "omega3..6 = 1",
                   "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic_for(args.workload, launch_bytes)},
        "cpu_baseline": cpu,
        "stream_copy_GB_per_s": copy["GB_per_s"],
        "variants": variants,
        "paper_context": {"RAFSINE_D3Q19_BGK_D3Q6_V100_MNUPS": 1307,
                          "VirtualFluids_D3Q27_cumulant_FCM_V100_MNUPS": 1064},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
