"""Benchmark: differentiable MLS-MPM sand digging, forward + backward, on one GPU.

One step = one full pass of the hot path over the batch: init state, a
500-sub-step recorded rollout (P2G with the SVD / Drucker-Prager update, grid
update with shovel contact, G2P, periodic binning, checkpoints), the loss,
and the reverse pass (segment recompute + adjoint of every sub-step).  The
rollout records its last checkpoint segments whole, as many as device memory
holds next to the rest of the workspace, so the reverse pass recomputes only
the segments before them (--record-segments).

Workload (default): batched system identification, 64 instances on 64^3
grids with particle counts uniform in [20k, 200k] (seeded), log-uniform E in
[1e4, 1e6] Pa, nu in [0.2, 0.4], friction angle in [20, 45] deg, 500 sub-steps
fwd+bwd, FP32, checkpoints every 50 sub-steps, binning interval autotuned.
Other workloads: the 64^3 dig with 1000 sub-steps fwd+bwd (dig3d_bwd) and the
128^3 cohesive bed with 2000 sub-steps fwd+bwd and its peak memory (dig3d_large).

Prints one JSON line (rank 0).  `value` is the batched fwd+bwd particle-steps/s
(eager launches, every kernel bracketed by HIP events); the same pass replayed
from a captured HIP graph, the plain per-instance loop on the same GPU and the
FP32-vs-FP64 gradient gate are reported beside it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "particle-steps/s fwd+bwd, batched vs plain, at grad rel-err <=1e-3 vs FP64"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sysid64",
                    choices=["sysid64", "dig3d_bwd", "dig3d_large", "optim", "dig3d_fwd", "sysid64_fwd",
                             "column2d_fwd"])
    ap.add_argument("--sub-steps", type=int, default=None, help="override rollout length (testing only)")
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"],
                    help="arithmetic of the fwd+bwd workloads; the gradient gate compares with FP64 (for an FP64 "
                         "run: another FP64 run binned every sub-step, a different order of the atomic sums)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-gate", action="store_true")
    ap.add_argument("--sort-every", type=int, default=0,
                    help="binning interval; 0 = autotune the batched context (the plain loop uses the same)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--streams", type=int, default=2,
                    help="contexts run at once for the headline pass (StreamGroup: the instances in groups of "
                         "balanced particle count, one stream each, graph-replayed); 1 = the single context")
    ap.add_argument("--treat", default="none", choices=["none", "clip", "scale", "norm", "record"],
                    help="gradient treatment inside the reverse pass (Sec. III-E) at the paper's thresholds; "
                         "'record' keeps the per-sub-step adjoint statistics without treating")
    ap.add_argument("--record-segments", type=int, default=0,
                    help="checkpoint segments the rollout records whole for the reverse pass (fewer replays); "
                         "0 = as many as fit in device memory with 16 GiB to spare")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB device copy (calibrates the HBM byte counters)")
    return ap.parse_args()


def build_batch(args):
    if args.workload == "dig3d_fwd":
        ws = [W.dig_3d(steps=500)]
        name = "dig3d_fwd: 64^3 dig, 219488 particles, 500 sub-steps forward, FP32"
    elif args.workload == "sysid64_fwd":
        ws = W.sysid_batch(64, steps=500)
        name = "sysid64_fwd: 64 instances, 64^3, N_i~U[20k,200k], 500 sub-steps forward, FP32"
    elif args.workload == "column2d_fwd":
        ws = [W.column_2d()]
        name = "column2d_fwd: 2D column collapse, 64^2, 2432 particles, 200 sub-steps forward, FP64"
    elif args.workload == "sysid64":
        ws = W.sysid_batch(64, steps=500)
        name = "sysid64: 64 instances, 64^3, N_i~U[20k,200k], 500 sub-steps fwd+bwd, K=50, FP32"
    elif args.workload == "dig3d_bwd":
        ws = [W.dig_3d_backward()]
        name = "dig3d_bwd: 64^3, 219488 particles, 1000 sub-steps fwd+bwd, K=50, FP32"
    else:
        ws = [W.dig_3d_large()]
        name = "dig3d_large: 128^3 cohesive bed, 1802416 particles, 2000 sub-steps fwd+bwd, K=100, FP32"
    if args.sub_steps:
        for w in ws:
            w.steps = args.sub_steps
    return ws, name


class Pass:
    """One context over a list of instances and the inputs of a full pass
    (init, recorded rollout, loss, backward: one ddm_pass call)."""

    def __init__(self, ddm, ws, sort_every, precision=None, stream=None, record_segments=1, grid_record_blocks=0):
        self.ws = ws
        self.steps = ws[0].steps
        cfg, insts = configs(ddm, ws, sort_every, precision, record_segments, grid_record_blocks)
        self.sim = ddm.Simulator(cfg, insts, stream=stream)
        # inputs resident in device memory, in the context's precision, before any timed pass
        torch = self.sim.torch
        self.x0 = torch.as_tensor(np.concatenate([W.bed_positions(w) for w in ws]),
                                  device=self.sim.device).to(self.sim.dtype)
        self.tg = torch.as_tensor(np.stack([W.target_heightmap(w) for w in ws]), device=self.sim.device)

    def run(self, graph=False):
        return self.sim.full_pass(self.x0, self.steps, self.tg, graph=graph)

    @property
    def particle_steps(self):
        return sum(w.n_particles for w in self.ws) * self.steps


def configs(ddm, ws, sort_every, precision=None, record_segments=1, grid_record_blocks=0):
    K = ws[0].checkpoint_every or 50
    cfgs = [ddm.from_workload(w, max_steps=ws[0].steps, checkpoint_every=K, precision=precision,
                              sort_every=sort_every) for w in ws]
    cfg = cfgs[0][0]
    cfg.record_segments = record_segments
    cfg.grid_record_blocks = grid_record_blocks
    return cfg, [c[1] for c in cfgs]


def pick_record_segments(ddm, torch, ws, sort_every, spare=16 << 30, precision=None, grid_record_blocks=0):
    """The most checkpoint segments whose whole record fits in free device
    memory next to the rest of the workspace, with `spare` bytes left over."""
    free = torch.cuda.mem_get_info()[0]
    K = ws[0].checkpoint_every or 50
    best = 1
    for m in range(1, (ws[0].steps + K - 1) // K + 1):
        cfg, insts = configs(ddm, ws, sort_every, precision, record_segments=m, grid_record_blocks=grid_record_blocks)
        if ddm.workspace_query(cfg, insts).workspace_bytes + spare <= free:
            best = m
    return best


def algorithmic_bytes_p2g(n_particles, n_active, b=4, d=3):
    """P2G moves per particle the state it reads (x, v, C, G: (2d + 2d^2) b) and
    the G' it writes (d^2 b); per active grid node (m > 0) the (d + 1) b it adds."""
    per_particle = (2 * d + 2 * d * d) * b + d * d * b
    return n_particles * per_particle + n_active * (d + 1) * b


def algorithmic_bytes_pass(n_particles, n_active, b=4, d=3):
    """Bytes per particle-step that a fwd+bwd pass must move: per particle the
    state written and read in the forward (2 S_p), again in the recompute
    (2 S_p), read once more in the reverse step (S_p) and the adjoint read and
    written (2 S_p), S_p = (2d + 2d^2) b; per active node (m > 0), in the
    forward, the recompute and the reverse step, m and mv written and read
    (2 (1 + d) b) and v written and read (2 d b)."""
    s_p = (2 * d + 2 * d * d) * b
    return 7 * s_p + 3 * (2 * (1 + d) * b + 2 * d * b) * n_active / n_particles


def algorithmic_bytes_forward(n_particles, n_active, b=4, d=3):
    """Bytes per particle-step of the forward sub-step: the state read and
    written (2 S_p) and, per active node, m and mv written and read and v
    written and read."""
    s_p = (2 * d + 2 * d * d) * b
    return 2 * s_p + (2 * (1 + d) * b + 2 * d * b) * n_active / n_particles


def active_nodes(sim, x0, steps, samples=10, blocks=False):
    """Mean number of grid nodes with m > 0 over a forward run of `steps`
    sub-steps from x0 (all instances), sampled every steps/samples sub-steps
    from the library's grid of the last sub-step.  blocks: also the largest
    sampled number of active blocks (4^dim nodes the grid update processed)."""
    sim.init_state(x0)
    every = max(1, steps // samples)
    counts, nblk, done = [], [], 0
    npb = 4 ** sim.dim
    while done < steps:
        k = min(every, steps - done)
        sim.step(k)
        done += k
        g = sim.get_grid()
        counts.append(int((g[:, :, 0] > 0).sum().item()))
        nblk.append(int(round((g[:, :, 7] > 0).sum().item() / npb)))
        del g
    if blocks:
        return float(np.mean(counts)), counts, max(nblk)
    return float(np.mean(counts)), counts


def grid_record_capacity(ddm, torch, ws, sort_every, precision=None):
    """Capacity of the pre-update grid record (blocks per sub-step): 1.5x the
    most active blocks sampled over a forward run of the workload (a smaller
    record leaves room for more recorded segments), with the mean active-node
    count of that run."""
    cfg, insts = configs(ddm, ws, sort_every, precision, record_segments=1)
    sim = ddm.Simulator(cfg, insts)
    x0 = np.concatenate([W.bed_positions(w) for w in ws])
    n_act, samples, most = active_nodes(sim, x0, ws[0].steps, blocks=True)
    del sim
    torch.cuda.empty_cache()
    return int(np.ceil(1.5 * most)), most, n_act, samples


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "p2g_sysid64_traffic.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2510_17335_amd", "csrc", "ddm_kernels.hip")


def measured_traffic(forward=False):
    """HBM bytes per P2G launch from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE per dispatch, each scaled by what the same counter reads for a
    plain copy of known size): of a launch of the recorded pass (which also
    keeps the stress for the reverse pass), or of a forward-only launch.  None
    when the summary is absent or the kernel source has changed since the
    counters were taken."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    try:
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
        if rec.get("kernel_source_sha256") != sha:
            return None
        copy_bytes = float(rec["copy_bytes"])
        f_fac = copy_bytes / (float(rec["copy_fetch_kib"]) * 1024)
        w_fac = copy_bytes / (float(rec["copy_write_kib"]) * 1024)
        pre = "p2g_forward_" if forward else "p2g_"
        return (float(rec[pre + "fetch_kib"]) * f_fac + float(rec[pre + "write_kib"]) * w_fac) * 1024
    except (KeyError, ValueError):
        return None


def fwd_traffic_applies(args):
    """The forward-only counters were taken on the 64-instance FP32 batch."""
    return args.workload == "sysid64_fwd" and args.precision == "f32"


def pass_traffic_applies(args):
    """The pass counters were taken on the 64-instance FP32 batch, untreated."""
    return args.workload == "sysid64" and args.precision == "f32" and args.treat == "none"


def copy_calibration(torch):
    """A plain device copy of 1 GiB (read 1 GiB, write 1 GiB), three times."""
    n = 1 << 28
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    print(f"# copy calibration: 3 x {4 * n} bytes read + written (elementwise neg)", flush=True)
    del src, dst


def host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count(), len(os.sched_getaffinity(0))


def cpu_baseline(ws, grad=True, target_s=15.0):
    """The FP64 oracle on one host core (pinned with sched_setaffinity) on the
    smallest instance of the workload, for about `target_s` seconds of work:
    with its 9 forward-mode tangents (the fwd+bwd-equivalent rate) when grad,
    else the plain FP64 forward."""
    import oracle
    oracle.build(force=False)
    w = min(ws, key=lambda q: q.n_particles)
    cfg = oracle.config(w)
    s0 = oracle.initial_state(W.bed_positions(w))
    tgt = W.target_heightmap(w) if grad else None
    old = os.sched_getaffinity(0)
    core = min(old)
    os.sched_setaffinity(0, {core})
    try:
        # a short run (doubled until it takes 0.5 s) sizes the sample: the
        # rollout's first sub-steps, up to the workload's length, repeated to
        # fill about target_s
        n = 1
        while True:
            t0 = time.perf_counter()
            oracle.rollout(cfg, w.params, s0, n, target=tgt, grad=grad)
            dt = time.perf_counter() - t0
            if dt >= 0.5 or n >= w.steps:
                break
            n = min(2 * n, w.steps)
        rate = w.n_particles * n / dt
        steps = int(min(w.steps, max(1, round(target_s * rate / w.n_particles))))
        reps = max(1, int(round(target_s * rate / (w.n_particles * steps))))
        t0 = time.perf_counter()
        for _ in range(reps):
            oracle.rollout(cfg, w.params, s0, steps, target=tgt, grad=grad)
        dt = time.perf_counter() - t0
    finally:
        os.sched_setaffinity(0, old)
    model, ncpu, navail = host_cpu()
    kind = "FP64 with 9 forward-mode tangents" if grad else "FP64 forward"
    return {"value": w.n_particles * steps * reps / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"smallest instance ({w.n_particles} particles), {reps} x {steps} sub-steps from its initial "
                      f"state, {kind}, {dt:.1f} s, pinned to core {core}",
            "host_cpu": model, "host_nproc": ncpu, "host_cpus_available": navail}


def stream_group_bench(args, torch, ddm, ws, R, TW, spare=16 << 30):
    """The batch as args.streams contexts at once (ddm.StreamGroup), each
    group's passes graph-replayed on its own stream: per group, a grid record
    of 1.5x its most active blocks (its own forward run) and the most segment
    sets that fit for all groups together with `spare` bytes left.  Returns
    (particle-steps/s, ms per pass, a config record, the gradients in the
    original instance order)."""
    S = args.streams
    groups = ddm.balanced_groups([w.n_particles for w in ws], S)
    caps = []
    for g in groups:
        cap_g, _, _, _ = grid_record_capacity(ddm, torch, [ws[i] for i in g], R, args.precision)
        caps.append(cap_g)
    free = torch.cuda.mem_get_info()[0]
    K = ws[0].checkpoint_every or 50
    M = 1
    for m in range(1, (ws[0].steps + K - 1) // K + 1):
        need = 0
        for g, cap_g in zip(groups, caps):
            cfg_g, insts_g = configs(ddm, [ws[i] for i in g], R, args.precision, record_segments=m,
                                     grid_record_blocks=cap_g)
            need += ddm.workspace_query(cfg_g, insts_g).workspace_bytes
        if need + spare <= free:
            M = m
    cfg, insts = configs(ddm, ws, R, args.precision)
    cfg.tile_workgroups = TW
    sg = ddm.StreamGroup(cfg, insts, groups, record_segments=[M] * len(groups), grid_record_blocks=caps)
    dev = torch.device("cuda:0")
    x0 = torch.as_tensor(np.concatenate([W.bed_positions(w) for w in ws]), device=dev)
    tg = torch.as_tensor(np.stack([W.target_heightmap(w) for w in ws]), device=dev)
    steps = ws[0].steps
    sg.set_inputs(x0, tg)                     # split once: the inputs stay in the groups' buffers
    for _ in range(max(1, args.warmup)):      # the first captures each group's pass
        sg.run(steps)
        sg.join()
    torch.cuda.synchronize()
    err = sg.check()
    if err.flags:
        raise RuntimeError(f"stream group: device flags {err.flags}")
    # every step joins the groups: the next step's passes wait for all of the
    # previous step's, as an optimiser step that reads every gradient would
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sg.run(steps)
        sg.join()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    loss, grad = sg.results()
    err = sg.check()
    work = sum(w.n_particles for w in ws) * steps
    value = work * args.steps / elapsed
    ms = 1e3 * elapsed / args.steps
    # the same passes with no join between steps: each group queues behind
    # its own previous pass only (independent instances)
    k_unjoined = min(args.steps, 3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(k_unjoined):
        sg.run(steps)
    sg.results()
    torch.cuda.synchronize()
    pipelined = work * k_unjoined / (time.perf_counter() - t0)
    err2 = sg.check()
    rec = {"contexts": len(groups), "particles": [sum(ws[i].n_particles for i in g) for g in groups],
           "record_segments": M, "grid_record_blocks": caps, "ms_per_step": ms,
           "unjoined_value": pipelined, "device_flags": int(err.flags | err2.flags)}
    print(f"# {len(groups)} contexts at once (graph-replayed): {ms:.1f} ms/step, {value:.3e} particle-steps/s, "
          f"{M} segment sets each, grid records {caps}; without a join between steps {pipelined:.3e}", flush=True)
    grads = grad.cpu().numpy()
    del sg
    return value, ms, rec, grads


def treatment_kwargs(args, steps):
    """Simulator.set_grad_treatment arguments for --treat (None for none)."""
    if args.treat == "none":
        return None
    if args.treat == "record":
        return {"mode": "none", "record_steps": steps}
    return {"mode": args.treat}


def optimiser_bench(args, torch, ddm):
    """Skill optimisation on the 64^3 dig (500 sub-steps, FP32): RMSprop with
    the 5-candidate line search, every iteration one fwd+bwd pass and one
    batched forward of the 5 candidates.  Reports iterations per second."""
    from paper_2510_17335_amd import optim as O
    w = W.dig_3d(steps=args.sub_steps or 500)
    x0, tg = W.bed_positions(w), W.target_heightmap(w)
    ev = O.GpuEvaluator(ddm, w, x0, tg, w.steps, checkpoint_every=50, treatment=treatment_kwargs(args, w.steps))
    spec = O.OptimSpec(free=["depth", "angle_deg", "push"], step=O.skill_steps())
    O.optimise(w.params, spec, ev.grad, ev.losses, max(1, args.warmup))      # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = O.optimise(w.params, spec, ev.grad, ev.losses, args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    n = sum(w.n_particles for _ in range(1)) * w.steps
    out = {"metric": "optimiser iterations/s (skill optimisation, 1 fwd+bwd pass + 5 batched candidate forwards)",
           "value": args.steps / el, "unit": "iterations/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic (seeded bed and target, no dataset)",
           "config": {"workload": f"optim: dig3d 64^3, {w.n_particles} particles, {w.steps} sub-steps, free depth/angle/push",
                      "grad_treatment": args.treat,
                      "particle_steps_per_iteration": n * 6},
           "losses": [h["loss"] for h in st.history], "chosen_alpha": [O.LINE_SEARCH[h["chosen"]] for h in st.history]}
    print(json.dumps(out), flush=True)


def forward_bench(args, torch, ddm):
    """Forward sub-steps only (Algorithm 1, no recording, no reverse pass): one
    step = init + the workload's sub-steps over the whole batch."""
    ws, wname = build_batch(args)
    prec = ws[0].precision
    b, d, steps = (8 if prec == "f64" else 4), ws[0].dim, ws[0].steps
    n = sum(w.n_particles for w in ws)
    print(f"# workload {wname}: {len(ws)} instances, {n} particles", flush=True)
    x0 = np.concatenate([W.bed_positions(w) for w in ws])
    sim = ddm.Simulator(*configs(ddm, ws, args.sort_every or 8), stream=torch.cuda.Stream())
    tuned = None
    if not args.sort_every:
        sim.init_state(x0)
        tuned = sim.autotune()
        print(f"# autotuned launch (binning interval, tile workgroups): {sim.launch()}", flush=True)
    R = tuned or args.sort_every
    TW = sim.launch()[1]
    n_act, samples = active_nodes(sim, x0, steps)
    print(f"# active grid nodes (m > 0), mean over the run: {n_act:.0f} (samples {samples})", flush=True)
    # positions resident in device memory, in the context's precision, before the timed region
    x0 = torch.as_tensor(x0, device=sim.device).to(sim.dtype)

    def one(s, x):
        s.init_state(x)
        s.step(steps)

    breakdown = None
    for i in range(args.warmup):
        last = i == args.warmup - 1
        if last:
            sim.set_timing(True)
        one(sim, x0)
        torch.cuda.synchronize()
        if last:
            breakdown = sim.read_timing()
            sim.set_timing(False)
        print(f"# warmup {i + 1}/{args.warmup} done", flush=True)
    # the timed region brackets only P2G (the roofline kernel) with events
    sim.set_timing(groups=["p2g"]) if breakdown else sim.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        one(sim, x0)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timing = sim.read_timing()
    sim.set_timing(False)
    breakdown = breakdown or timing
    err = sim.check()
    value = n * steps * args.steps / elapsed
    print(f"# batched forward: {1e3 * elapsed / args.steps:.2f} ms/step, {value:.3e} particle-steps/s, "
          f"device flags {err.flags}", flush=True)
    del sim
    torch.cuda.empty_cache()

    plain_value = None
    if len(ws) > 1 and not args.no_plain:
        t_plain = 0.0
        for w in ws:
            ps = ddm.Simulator(*configs(ddm, [w], R))
            xw = torch.as_tensor(W.bed_positions(w), device=ps.device).to(ps.dtype)
            one(ps, xw)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            one(ps, xw)
            torch.cuda.synchronize()
            t_plain += time.perf_counter() - t1
            del ps
        plain_value = n * steps / t_plain
        print(f"# plain loop: {t_plain * 1e3:.1f} ms/step, {plain_value:.3e} particle-steps/s", flush=True)

    p2g_ms, p2g_n = timing["p2g"]
    per_launch = algorithmic_bytes_p2g(n, n_act, b, d)
    achieved = per_launch / (p2g_ms / p2g_n * 1e-3) / 1e9 if p2g_n else None
    fwd_bytes = algorithmic_bytes_forward(n, n_act, b, d)
    bound = HBM_PEAK_GBS * 1e9 / fwd_bytes
    cpu = None if args.no_cpu else cpu_baseline(ws, grad=False)
    out = {
        "metric": "particle-steps/s forward (Algorithm 1 sub-steps), batched vs plain",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": prec, "data": "synthetic (seeded beds, no dataset)",
        "config": {"workload": wname, "instances": len(ws), "particles": n, "sub_steps": steps,
                   "sort_every": R, "sort_every_autotuned": tuned is not None, "plain_sort_every": R,
                   "tile_workgroups": TW, "active_nodes_mean": n_act},
        "plain_value": plain_value,
        "batched_over_plain": (value / plain_value) if plain_value else None,
        "kernel_ms": {k: {"ms": round(v[0], 3), "launches": v[1]} for k, v in breakdown.items() if v[1]},
        "kernel_ms_from": "last warm-up run, every launch group timed" if args.warmup else "timed region",
        "roofline": {"bound": "hbm", "kernel": "p2g", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                     "traffic": measured_traffic(forward=True) if fwd_traffic_applies(args) else None,
                     "algorithmic_bytes": per_launch},
        "pass_roofline": {"bytes_per_particle_step": fwd_bytes, "bound_value": bound, "unit": "particle-steps/s",
                          "frac": value / bound},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2510_17335_amd as ddm
    if args.workload == "optim":
        optimiser_bench(args, torch, ddm)
        return
    if args.workload.endswith("_fwd"):
        forward_bench(args, torch, ddm)
        return
    assert torch.cuda.is_available(), "needs a GPU"
    dev = torch.device("cuda:0")
    if args.copy_calib:
        copy_calibration(torch)
    ws, wname = build_batch(args)
    print(f"# workload {wname}: {len(ws)} instances, {sum(w.n_particles for w in ws)} particles", flush=True)

    # batched: one context on its own stream, binning interval autotuned on the
    # initial state (unless --sort-every is given).  A forward run first counts
    # the active grid nodes and blocks: the record of each sub-step's
    # pre-update grid holds 1.5x the most active blocks seen (fewer bytes per
    # recorded segment, so more segments fit).
    cap, most, n_act, act_samples = grid_record_capacity(ddm, torch, ws, args.sort_every or 32, args.precision)
    for attempt in range(2):
        rseg = args.record_segments or pick_record_segments(ddm, torch, ws, args.sort_every or 8,
                                                            precision=args.precision, grid_record_blocks=cap)
        print(f"# checkpoint segments recorded by the rollout: {rseg} (pre-update grid record: "
              f"{cap or 'every'} blocks per sub-step; most active blocks sampled: {most})", flush=True)
        bp = Pass(ddm, ws, args.sort_every or 8, precision=args.precision, stream=torch.cuda.Stream(),
                  record_segments=rseg, grid_record_blocks=cap)
        treat = treatment_kwargs(args, ws[0].steps)
        if treat:
            bp.sim.set_grad_treatment(**treat)
        tuned = None
        if not args.sort_every:
            bp.sim.init_state(bp.x0)
            tuned = bp.sim.autotune()
            print(f"# autotuned launch (binning interval, tile workgroups): {bp.sim.launch()}", flush=True)
        R = tuned or args.sort_every
        TW = bp.sim.launch()[1]
        n_part = sum(w.n_particles for w in ws)
        print(f"# active grid nodes (m > 0), mean over the forward run: {n_act:.0f} (samples {act_samples})",
              flush=True)
        breakdown = None
        for i in range(args.warmup):
            last = i == args.warmup - 1
            if last:
                bp.sim.set_timing(True)
            bp.run()
            torch.cuda.synchronize()
            if last:
                breakdown = bp.sim.read_timing()
                bp.sim.set_timing(False)
            print(f"# warmup {i + 1}/{args.warmup} done", flush=True)
        try:
            bp.sim.check()
            break
        except ddm.DdmError as e:
            if e.code != ddm.DDM_ENOMEM or cap == 0:
                raise
            # a sub-step had more active blocks than the record holds: every block then
            print(f"# {e}; again with a record of every block", flush=True)
            del bp
            torch.cuda.empty_cache()
            cap = 0
    bp.sim.check()
    torch.cuda.reset_peak_memory_stats()
    # the timed region brackets only P2G (the roofline kernel) with events: an
    # event pair per launch of every group would cost about 35 ms per pass
    bp.sim.set_timing(groups=["p2g"]) if breakdown else bp.sim.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        loss, grad = bp.run()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    peak_gb = torch.cuda.max_memory_allocated() / 1e9
    timing = bp.sim.read_timing()
    bp.sim.set_timing(False)
    err = bp.sim.check()
    ms_per_step = 1e3 * elapsed / args.steps
    value = bp.particle_steps * args.steps / elapsed
    print(f"# batched: {ms_per_step:.1f} ms/step, {value:.3e} particle-steps/s, device flags {err.flags}",
          flush=True)
    grads32 = grad.cpu().numpy()

    # the same pass captured once into a HIP graph and replayed (not the timed
    # region above: per-kernel events cannot sit inside a graph)
    graph_value = None
    if not args.no_graph:
        bp.run(graph=True)
        torch.cuda.synchronize()
        tg0 = time.perf_counter()
        for i in range(args.steps):
            bp.run(graph=True)
        torch.cuda.synchronize()
        graph_value = bp.particle_steps * args.steps / (time.perf_counter() - tg0)
        print(f"# graph replay: {graph_value:.3e} particle-steps/s", flush=True)

    # dominant kernel group (from the warm-up pass that timed every group) and
    # the roofline of P2G (bytes moved per launch / its launch time measured
    # in the timed region)
    breakdown = breakdown or timing
    dom = max(breakdown, key=lambda k: breakdown[k][0])
    p2g_ms, p2g_n = timing["p2g"]
    esz = 8 if args.precision == "f64" else 4
    per_launch_bytes = algorithmic_bytes_p2g(n_part, n_act, b=esz)
    achieved = per_launch_bytes / (p2g_ms / p2g_n * 1e-3) / 1e9 if p2g_n else None
    breakdown = {k: {"ms": round(v[0], 3), "launches": v[1]} for k, v in breakdown.items() if v[1]}

    # the batched context's workspace (up to most of the device) goes before
    # the plain loop and the FP64 gate allocate theirs
    del bp
    torch.cuda.empty_cache()

    # the headline: the same batch as args.streams contexts at once
    streams_value, streams_ms, streams_cfg = None, None, None
    if args.streams > 1 and len(ws) >= args.streams and args.treat == "none":
        try:
            streams_value, streams_ms, streams_cfg, grads_s = stream_group_bench(args, torch, ddm, ws, R, TW)
        except (ddm.DdmError, torch.cuda.OutOfMemoryError) as e:
            if isinstance(e, ddm.DdmError) and e.code != ddm.DDM_ENOMEM:
                raise
            # out of device memory: the line then reports the single context (the same work)
            print(f"# {args.streams} contexts at once: not run ({e})", flush=True)
            streams_cfg = {"contexts": args.streams, "error": str(e)}
        else:
            rel = np.abs(grads_s - grads32) / np.maximum(np.abs(grads32), 1e-6 * np.abs(grads32).max())
            streams_cfg["grad_rel_diff_vs_single_context"] = float(rel.max())
        torch.cuda.empty_cache()

    plain_value = None
    if not args.no_plain:
        t_plain = 0.0
        for w in ws:
            pp = Pass(ddm, [w], R, precision=args.precision, record_segments=rseg)
            pp.run()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            pp.run()
            torch.cuda.synchronize()
            t_plain += time.perf_counter() - t1
            del pp
        plain_value = sum(w.n_particles for w in ws) * ws[0].steps / t_plain
        print(f"# plain loop: {t_plain * 1e3:.1f} ms/pass, {plain_value:.3e} particle-steps/s", flush=True)
        torch.cuda.empty_cache()

    gate = None
    if not args.no_gate:
        # the batched gradients of the two smallest instances against the FP64 path
        idx = sorted(range(len(ws)), key=lambda i: ws[i].n_particles)[:2]
        rels, per_param = [], []
        for i in idx:
            p64 = Pass(ddm, [ws[i]], 1 if args.precision == "f64" else 8, precision="f64")
            _, g64 = p64.run()
            g64 = g64[0].cpu().numpy()
            scale = np.abs(g64).max()
            rel = np.abs(grads32[i] - g64) / np.maximum(np.abs(g64), 1e-6 * scale)
            rels.append(float(rel[np.abs(g64) > 1e-6 * scale].max()))
            per_param.append([float(f"{r:.2g}") for r in rel])
            del p64
        gate = {"instances": idx, "max_rel_err": max(rels), "pass": max(rels) <= 1e-3,
                "rel_err_per_param": dict(zip(ddm.PARAM_NAMES, per_param[int(np.argmax(rels))]))}
        print(f"# gradient gate ({args.precision} vs FP64): {gate}", flush=True)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(ws)
        # the oracle's plain FP64 forward as well (no tangents), a shorter sample
        fwd = cpu_baseline(ws, grad=False, target_s=5.0)
        cpu["forward_value"] = fwd["value"]
        cpu["forward_sample"] = fwd["sample"]
    # the whole pass against the HBM roofline of its algorithmic bytes
    pass_bytes = algorithmic_bytes_pass(n_part, n_act, b=esz)
    pass_bound = HBM_PEAK_GBS * 1e9 / pass_bytes
    single_value, single_ms = value, ms_per_step
    if streams_value:
        value, ms_per_step = streams_value, streams_ms
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic (seeded beds and targets, no dataset)",
        "config": {"workload": wname, "instances": len(ws), "particles": sum(w.n_particles for w in ws),
                   "sub_steps": ws[0].steps, "checkpoint_every": ws[0].checkpoint_every,
                   "sort_every": R, "sort_every_autotuned": tuned is not None, "plain_sort_every": R,
                   "tile_workgroups": TW, "active_nodes_mean": n_act,
                   "record_segments": rseg, "grid_record_blocks": cap, "active_blocks_max_sampled": most,
                   "grad_treatment": args.treat,
                   "peak_mem_gb": round(peak_gb, 2)},
        "headline": (f"{args.streams} contexts at once, graph-replayed passes" if streams_value
                     else "one context, eager launches"),
        "single_context_value": single_value,
        "single_context_ms_per_step": single_ms,
        "graph_value": graph_value,
        "streams": streams_cfg,
        "plain_value": plain_value,
        "batched_over_plain": (value / plain_value) if plain_value else None,
        "grad_gate": gate,
        "kernel_ms": breakdown,
        "kernel_ms_from": "last warm-up pass, every launch group timed" if args.warmup else "timed region",
        "roofline": {"bound": "hbm", "kernel": "p2g", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                     "traffic": measured_traffic() if pass_traffic_applies(args) else None,
                     "algorithmic_bytes": per_launch_bytes,
                     "dominant_group": dom},
        "pass_roofline": {"bytes_per_particle_step": pass_bytes, "bound_value": pass_bound, "unit": "particle-steps/s",
                          "frac": value / pass_bound},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
