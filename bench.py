"""Benchmark: forward + backward differentiable-PD time steps per second on one
MI355X.

Default workload (--config batch): the identification batch, 64 uneven scenes
(beams and anchored blobs, 1k-30k tets each, about 0.73 M tets in total, FP64)
stepped together; the loss is trajectory matching, sum over steps of the
mass-weighted distance to an observed trajectory that another material field
generated, and its gradient goes to every tet's log E.  One bench step = one
batched time step of every scene solved forward to the dual gate (1e-6) plus
its adjoint step (trust-region selection, filtered prox differential, adjoint
solve, gradient routing).  The timed region runs K forward steps (with
checkpoints) and then the K backward steps, all inputs resident in HBM.
`--config c2` runs the single 20,000-tet heterogeneous beam instead, `drop`
the contact drop, `warmstart` the learned start on held-out drops.  Prints ONE
JSON line.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd PD steps/sec at 1e-6 residual (plain vs warm-started); % HBM roofline"
# adjoint tolerance of the benchmarked steps: the loosest PCG stop whose
# gradients stay within 1e-6 (relative) of the oracle's on the heterogeneous
# beam (tests/test_gpu_hetero_beam.py checks exactly this setting)
ADJ_TOL = 1e-10
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6

# kernel ids understood by pd_kernel_timer (see include/pdhot.h)
KERNELS = {"local": 0, "gather": 1, "top": 2, "bottom": 3, "Eb": 4, "apply_K": 5, "solve": 6}
CPU_BATCH_STEPS = 3  # steps of every batch scene in the CPU baseline
LEARNED_EDGE_WEIGHT = 100.0  # edge-difference weight of the warm-start network's training loss


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="batch")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=20)
    ap.add_argument("--timed-kernel", default="solve", choices=sorted(KERNELS))
    ap.add_argument("--max-sub", type=int, default=0)
    ap.add_argument("--iface-levels", type=int, default=0,
                    help="separator-tree levels of the interface solve (0: library default)")
    ap.add_argument("--no-warm-run", action="store_true", help="skip the warm-started measurements")
    ap.add_argument("--train-scenes", type=int, default=4, help="beams the warm-start network is trained on")
    ap.add_argument("--train-epochs", type=int, default=32)
    ap.add_argument("--batch-scenes", type=int, default=64, help="scenes of --config batch")
    ap.add_argument("--tune-cache", default="", help="autotuner cache file of --config batch")
    ap.add_argument("--drop-res", type=int, default=27, help="cells along the blob of --config drop (27: 28k tets)")
    ap.add_argument("--friction", type=float, default=0.5, help="Coulomb coefficient of the obstacles of --config drop")
    ap.add_argument("--energy", type=int, default=-1, choices=[-1, 0, 1, 2],
                    help="energy of a single-scene configuration: 0 Neo-Hookean prox, 1 corotated + volume "
                         "composite, 2 logarithmic volume barrier (-1: the configuration's own)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy a 64 MiB device buffer 3 times (calibrates the HBM byte counters) and exit")
    return ap.parse_args()


# committed counter summaries of the workloads that have one
TRAFFIC_FILES = {("c2", None): "traffic_solve_and_local_kernels_hetero_beam_20k_tets.txt",
                 ("drop", 41): "traffic_interface_solve_contact_drop_100k_tets.txt",
                 ("batch", None): "traffic_solve_identification_batch_64_scenes.txt"}


def measured_traffic(kernel, config="c2", drop_res=None):
    """DRAM bytes per working launch of `kernel` from the committed counter
    summary of this workload (FETCH_SIZE / WRITE_SIZE passes scaled by a copy
    of known size), or None when the workload or the kernel has none."""
    name = TRAFFIC_FILES.get((config, drop_res if config == "drop" else None))
    if name is None:
        return None
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic_per_working_launch_bytes:"):
            _, k, v = line.split()
            if k == kernel:
                return int(v)
    return None


def ensure_built():
    from paper_2605_14526_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2605_14526_amd import build
        build.build()


def rollout_fwd_bwd(g, sc, K, torch, dev, net=None, logw=None):
    """K forward steps with checkpoints, then K backward steps.  With a
    warm-start network, each step starts from its prediction (its inference is
    inside the timed region)."""
    q = dev(sc.q0())
    v = dev(sc.v0())
    g.contact_hist, g.active_hist = [], []
    forces = [dev(sc.f_ext(t)) for t in range(K)]
    ckpts = [g.new_ckpt() for _ in range(K)]
    qs = [torch.empty_like(q) for _ in range(K + 1)]
    vs = [torch.empty_like(q) for _ in range(K + 1)]
    qs[0].copy_(q)
    vs[0].copy_(v)
    g_logE = torch.zeros(sc.n_e, dtype=torch.float64, device="cuda")
    gq_t, gv_t, gf = torch.empty_like(q), torch.empty_like(q), torch.empty_like(q)
    target = torch.tensor(sc.target_centroid, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fiters, biters = [], []
    q0 = torch.empty_like(q) if net is not None else None
    for t in range(K):
        if net is not None:
            net.forward(qs[t], vs[max(t - 1, 0)], vs[t], forces[t], logw, q0=q0)
        _, _, st = g.step_forward(qs[t], vs[t], forces[t], q0=q0, q_next=qs[t + 1], v_next=vs[t + 1], ckpt=ckpts[t])
        fiters.append(st["iters"])
        g.contact_hist.append(st["n_contacts"])
        g.active_hist.append(st["n_active"])
    # loss = |mean(q_K) - target|^2 (the gradient is formed on the device)
    c = qs[K].mean(dim=0)
    gq = (2.0 * (c - target) / sc.n_v).expand_as(qs[K]).contiguous()
    gv = torch.zeros_like(gq)
    g.adjoint_reset()
    for t in reversed(range(K)):
        g.step_backward(ckpts[t], gq, gv, g_logE=g_logE, gq_t=gq_t, gv_t=gv_t, gf_ext=gf)
        gq, gq_t = gq_t, gq
        gv, gv_t = gv_t, gv
        biters.append(g.last_bwd_stats["adj_iters"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return t1 - t0, fiters, biters, g_logE


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(samples, threads=None):
    """The FP64 CPU oracle on (scene, steps) samples of the same workload: each
    sample is a forward rollout of `steps` steps and its reverse sweep of the
    centroid loss.  Returns (seconds, scene-steps, threads used)."""
    import oracle as O
    from paper_2605_14526_amd import scenes
    n0 = O.get_threads()
    if threads:
        O.set_threads(threads)
    used = O.get_threads()
    busy = 0.0
    done = 0
    try:
        for sc, steps in samples:
            osc = O.OracleScene(sc, eps_adj=ADJ_TOL)  # setup and factorization are not timed
            t0 = time.perf_counter()
            if sc.obstacles and getattr(sc, "friction", 0.0) > 0.0:
                q, v, ck, _ = O.rollout_friction(osc, steps, sc.friction)
                _, gq = scenes.centroid_loss(q, sc.target_centroid)
                O.rollout_backward_friction(osc, ck, gq, np.zeros_like(gq), sc.friction)
            elif sc.obstacles:
                q, v, ck, _ = O.rollout_contact(osc, steps)
                _, gq = scenes.centroid_loss(q, sc.target_centroid)
                O.rollout_backward_contact(osc, ck, gq, np.zeros_like(gq))
            else:
                q, v, ck, _ = O.rollout(osc, steps)
                _, gq = scenes.centroid_loss(q, sc.target_centroid)
                O.rollout_backward(osc, ck, gq, np.zeros_like(gq))
            busy += time.perf_counter() - t0
            done += steps
            print(f"[bench] cpu baseline ({used} threads): {sc.name} {steps} steps "
                  f"({busy:.1f} s)", file=sys.stderr, flush=True)
    finally:
        O.set_threads(n0)
    return busy, done, used


def cpu_baseline_entry(samples_all, samples_one, what):
    """cpu_baseline on all host threads and on one thread (a smaller sample)."""
    t, n, used = cpu_baseline(samples_all)
    t1, n1, _ = cpu_baseline(samples_one, threads=1)
    return {"value": round(n / t, 4), "unit": "scene fwd+bwd steps/s", "cores": used, "kind": "oracle",
            "sample": f"{what}: {n} scene-steps in {t:.2f} s on {used} threads (OpenMP over elements, fixed "
                      f"summation order, fixed-point adjoint to {ADJ_TOL:g})",
            "one_thread": {"value": round(n1 / t1, 4), "sample": f"{n1} scene-steps in {t1:.2f} s"},
            "host_cores": host_cores(), "cpu_model": cpu_model()}


def roofline_entry(kernel, bound, ms, launches, work, peak, unit, traffic=None, extra=None):
    achieved = work / (ms * 1e-3) / (1e9 if unit == "GB/s" else 1e12) if ms > 0 else 0.0
    r = {"kernel": kernel, "bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
         "frac": round(achieved / peak, 4), "traffic": traffic,
         "avg_launch_us": round(1000.0 * ms / max(launches, 1), 3), "launches": int(launches)}
    if extra:
        r.update(extra)
    return r


def profile_value(name, key):
    """A figure from a committed profile summary (`key: value` line), or None."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith(key + ":"):
            return float(line.split(":", 1)[1].split()[0])
    return None


def bench_batch(args, torch):
    """Identification batch (64 uneven beams and anchored blobs, about 0.73 M
    tets): batched fwd+bwd scene-steps per second of the trajectory-matching
    loss after autotuning the launch shapes."""
    from paper_2605_14526_amd import autotune, scenes
    from paper_2605_14526_amd.binding import Batch, Scene
    K = args.steps
    horizon = max(K, args.warmup, 2)
    scs = scenes.sysid_batch(n=args.batch_scenes, steps=50)
    t0 = time.perf_counter()
    gs = [Scene.from_scene(sc, eps_adj=ADJ_TOL, adj_warm=3, max_sub=args.max_sub, iface_levels=args.iface_levels)
          for sc in scs]
    t_setup = time.perf_counter() - t0
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")  # noqa: E731
    forces = [[dev(sc.f_ext(t)) for sc in scs] for t in range(horizon)]
    # 2 m_v per vertex and axis: the loss gradient 2 m (q_t - q_t^obs) over all scenes in three multi-tensor launches
    mass2 = [(2.0 * dev(g.vertex_mass())[:, None]).expand(sc.n_v, 3).contiguous() for g, sc in zip(gs, scs)]
    # observed trajectories: each scene rolled out with its observation field (setup, untimed)
    t0 = time.perf_counter()
    obs = []
    for g, sc in zip(gs, scs):
        g.set_material(sc.log_E_obs)
        g.factorize()
        q, v = dev(sc.q0()), dev(sc.v0())
        traj = [q]
        for t in range(horizon):
            q, v, _ = g.step_forward(q, v, forces[t][len(obs)])
            traj.append(q)
        obs.append(traj)
        g.set_material(sc.log_E)
        g.factorize()
    t_obs = time.perf_counter() - t0
    print(f"[bench] batch of {len(scs)} scenes set up in {t_setup:.1f} s, observations in {t_obs:.1f} s",
          file=sys.stderr, flush=True)
    B = Batch(gs)
    g_logE = [torch.zeros(sc.n_e, dtype=torch.float64, device="cuda") for sc in scs]

    q_init = [dev(sc.q0()) for sc in scs]
    v_init = [dev(sc.v0()) for sc in scs]

    def rollout(n, inertial=False):
        q, v = q_init, v_init
        traj, cks, fi, bi = [q], [], [], []
        loss = 0.0
        for t in range(n):
            ck = [g.new_ckpt() for g in gs]
            q0 = [qq + sc.h * vv for qq, vv, sc in zip(q, v, scs)] if inertial else None
            q, v, st, _ = B.step_forward(q, v, forces[t], q0=q0, ckpt=ck)
            traj.append(q)
            cks.append(ck)
            fi.append(np.mean([x["iters"] for x in st]))
        # trajectory loss sum_t sum_v m_v |q_t,v - q_t,v^obs|^2 (its gradient is formed on the device)
        def loss_grad(t):
            d = torch._foreach_sub(traj[t], [o[t] for o in obs])
            torch._foreach_mul_(d, mass2)
            return d
        gq = loss_grad(n)
        gv = [torch.zeros_like(x) for x in gq]
        for g in gs:
            g.adjoint_reset()
        torch._foreach_zero_(g_logE)
        for t in reversed(range(n)):
            gq, gv, _, _, st, _ = B.step_backward(cks[t], gq, gv, g_logE=g_logE)
            bi.append(np.mean([x["adj_iters"] for x in st]))
            if t > 0:
                gq = torch._foreach_add(gq, loss_grad(t))
        return fi, bi

    t1 = time.perf_counter()
    cfg = autotune.autotune(B, lambda: rollout(2), torch, cache_path=args.tune_cache or None, reps=1)
    t_tune = time.perf_counter() - t1
    # the solve is timed per launch inside the timed region; graphs carry no per-launch events
    if cfg.get("use_graph"):
        B.config(cfg["block_local"], cfg["block_applyK"], cfg["iters_per_check"], 0)
    rollout(args.warmup)
    B.kernel_timer(KERNELS["solve"])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    fi, bi = rollout(K)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t2
    s_ms, s_launch, s_bytes = B.kernel_timer_read()
    B.kernel_timer(-1)
    assert all(bool(torch.isfinite(x).all()) for x in g_logE)
    print(f"[bench] timed {K} batched fwd+bwd steps in {dt:.3f} s; fwd iters/scene-step {np.mean(fi):.2f}, "
          f"adjoint {np.mean(bi):.2f}", file=sys.stderr, flush=True)
    # the local step's FP64 rate over the same K steps (a separate run, not part of `value`)
    B.kernel_timer(KERNELS["local"])
    rollout(K)
    l_ms, l_launch, l_bytes = B.kernel_timer_read()
    B.kernel_timer(-1)
    ne = sum(sc.n_e for sc in scs)
    nnz = sum(g.factor_nnz() for g in gs)
    # inertial start q0 = q_t + h v_t, same gate
    fw = bw = None
    if not args.no_warm_run:
        rollout(min(args.warmup, 2), inertial=True)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        fw, bw = rollout(K, inertial=True)
        torch.cuda.synchronize()
        dtw = time.perf_counter() - t3
    prof = "fp64_counters_local_step_identification_batch_64_scenes.txt"
    flop_per_byte = profile_value(prof, "fp64_flop_per_algorithmic_byte")
    roof = roofline_entry("solve (interface right-hand side + interface solve + subdomain solve)", "hbm", s_ms,
                          s_launch, s_bytes, HBM_PEAK_GBS, "GB/s",
                          traffic=measured_traffic("solve", "batch"),
                          extra={"algorithmic_bytes": "per solve 16 B x nnz(L) of a nested-dissection Cholesky "
                                                      "factor of A~ + 6 x 24 B x n_free, summed over the solves "
                                                      "each scene did",
                                 "bytes_timed": round(s_bytes), "sum_nnz_L": round(nnz)})
    out = {"metric": METRIC, "value": round(len(scs) * K / dt, 3), "unit": "scene fwd+bwd steps/s",
           "n_gpus": 1, "steps": K, "warmup": args.warmup,
           "ms_per_step": round(1000.0 * dt / K, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"identification batch: {len(scs)} uneven scenes "
                                  f"({sum('blob' in sc.name for sc in scs)} anchored blobs, the rest beams), "
                                  f"{ne} tets in total (1k-30k each), contrast 1-100x, nu 0.40-0.49, h 0.01, "
                                  f"{K} batched steps, trajectory-matching loss against observations from "
                                  f"another material field, gradient w.r.t. every log E, gate 1e-6, "
                                  f"adjoint PCG to {ADJ_TOL:g}, plain q0 = q_t",
                      "launch_shapes": cfg, "setup_s": round(t_setup, 2), "tune_s": round(t_tune, 2),
                      "fwd_iters_per_step": round(float(np.mean(fi)), 3),
                      "adj_iters_per_step": round(float(np.mean(bi)), 3)},
           "roofline": roof,
           "roofline_local": roofline_entry(
               "local step (batched)", "fp64" if flop_per_byte else "hbm", l_ms, l_launch,
               l_bytes * flop_per_byte if flop_per_byte else l_bytes, FP64_VECTOR_PEAK_TFLOPS if flop_per_byte
               else HBM_PEAK_GBS, "TFLOP/s" if flop_per_byte else "GB/s",
               extra={"hbm_GBps": round(l_bytes / max(l_ms, 1e-9) / 1e6, 2),
                      "hbm_frac": round(l_bytes / max(l_ms, 1e-9) / 1e6 / HBM_PEAK_GBS, 4),
                      "flops": f"FP64 flops per algorithmic byte {flop_per_byte} from {prof}"
                      if flop_per_byte else None}),
           }
    if fw is not None:
        out["warm_started"] = {"inertial": {"value": round(len(scs) * K / dtw, 3), "unit": "scene fwd+bwd steps/s",
                                            "ms_per_step": round(1000.0 * dtw / K, 4),
                                            "fwd_iters_per_step": round(float(np.mean(fw)), 3),
                                            "adj_iters_per_step": round(float(np.mean(bw)), 3),
                                            "start": "q0 = q_t + h v_t"}}
    if not args.no_cpu_baseline:
        # every scene of the batch for its first CPU_BATCH_STEPS steps (about 10 s on 16 threads), and three
        # of them on one thread
        n = min(CPU_BATCH_STEPS, K)
        one = list(range(0, len(scs), 24))
        out["cpu_baseline"] = cpu_baseline_entry([(sc, n) for sc in scs], [(scs[i], n) for i in one],
                                                 f"first {n} fwd+bwd steps of all {len(scs)} scenes of the batch "
                                                 f"({ne} tets; one thread: scenes {one}), centroid loss")
    print(json.dumps(out), flush=True)


def bench_warmstart(args, torch):
    """The learned warm start on held-out contact scenes of other shapes: one network instance per mesh, all
    sharing one set of weights, trained on the GPU on plain rollouts of drops of `train_scenes` seeded blobs,
    then plain, inertial and learned starts on 10 held-out drops of 10 other seeded blobs (forward steps:
    the start only changes the forward iteration)."""
    from paper_2605_14526_amd import scenes, warmstart
    from paper_2605_14526_amd.binding import Mpn, Scene
    res, S = args.drop_res, args.steps
    fam = lambda k: scenes.shape_family(k, res=res, steps=100, friction=args.friction)  # noqa: E731
    t0 = time.perf_counter()
    train_sc = [fam(k) for k in range(args.train_scenes)]
    samples = []
    for k, sc in enumerate(train_sc):
        samples.append(warmstart.generate([sc], 100, torch))
        print(f"[bench] trajectories of training blob {k} ({sc.n_e} tets) in {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    t_gen = time.perf_counter() - t0
    nets = [Mpn.for_scene(sc, edge_weight=LEARNED_EDGE_WEIGHT) for sc in train_sc]
    master = nets[0]
    master.init_params(1)
    for n in nets[1:]:
        n.share_params(master)
    # RMS correction over every training mesh (each with its own free vertices)
    scale = float(np.sqrt(np.mean([warmstart.output_scale(ss, sc.h, sc.pinned) ** 2
                                   for ss, sc in zip(samples, train_sc)])))
    for n in nets:
        n.set_output_scale(scale)
    t0 = time.perf_counter()
    hist = warmstart.train_shared(master, nets, samples, args.train_epochs, lr=1e-3, seed=1, lr_decay=0.9)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    n_samples = sum(len(x) for x in samples)
    # the least-squares scale of the network's correction on the training samples
    alpha = warmstart.fit_correction_scale(nets, samples, train_sc[0].h, torch)
    scale *= alpha
    print(f"[bench] trained on {n_samples} samples of {len(train_sc)} blobs in {t_train:.1f} s "
          f"(trajectories {t_gen:.1f} s); correction scale {alpha:.3f}", file=sys.stderr, flush=True)
    res_rows = {"plain": [], "inertial": [], "learned": []}
    sizes = []
    for k in range(900, 910):
        sc = fam(k)
        sizes.append(sc.n_e)
        g = Scene.from_scene(sc)
        gi = Scene.from_scene(sc, fwd_start=1)
        net = Mpn.for_scene(sc, edge_weight=LEARNED_EDGE_WEIGHT)
        net.share_params(master)
        net.set_output_scale(scale)
        logw = torch.tensor(g.vertex_logw(), dtype=torch.float64, device="cuda")
        for start in ("plain", "inertial", "learned"):
            gg = gi if start == "inertial" else g
            warmstart.rollout(gg, sc, 2, torch, start=start, net=net, logw=logw)  # warm caches
            _, _, its, sec = warmstart.rollout(gg, sc, S, torch, start=start, net=net, logw=logw)
            res_rows[start].append((float(np.mean(its)), S / sec))
        print(f"[bench] held-out blob {k} ({sc.n_e} tets): " +
              ", ".join(f"{s_} {res_rows[s_][-1][0]:.2f} it" for s_ in res_rows), file=sys.stderr, flush=True)
        net.close()
        g.close()
        gi.close()
    summ = {s_: {"fwd_iters_per_step": round(float(np.mean([a for a, _ in v])), 3),
                 "fwd_steps_per_s": round(float(np.mean([b for _, b in v])), 2)} for s_, v in res_rows.items()}
    out = {"metric": METRIC, "value": summ["learned"]["fwd_steps_per_s"], "unit": "forward steps/s (learned start)",
           "n_gpus": 1, "steps": S, "warmup": 2, "ms_per_step": round(1000.0 / summ["learned"]["fwd_steps_per_s"], 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64 solve, bf16 network",
           "data": "synthetic",
           "config": {"workload": f"10 held-out drops of 10 other seeded blobs ({min(sizes)}-{max(sizes)} tets, "
                                  f"cells {res} along the largest extent, initial velocities seeded), {S} forward "
                                  f"steps each, gate 1e-6 and FB residual 1e-10 whatever the start",
                      "starts": summ,
                      "train": {"blobs": len(train_sc), "samples": n_samples, "epochs": args.train_epochs,
                                "generate_s": round(t_gen, 2), "train_s": round(t_train, 2),
                                "correction_scale": round(alpha, 4),
                                "final_loss": hist[-1], "weights": "one set shared by every mesh's instance"}}}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); this build has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_probe:
        n = 8 * 1024 * 1024
        x = torch.randn(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(f"[bench] copied 3 x {n * 8 >> 20} MiB", file=sys.stderr, flush=True)
        return
    ensure_built()
    if args.config == "batch":
        bench_batch(args, torch)
        return
    if args.config == "warmstart":
        bench_warmstart(args, torch)
        return
    from paper_2605_14526_amd import scenes
    from paper_2605_14526_amd.binding import Scene

    drop = args.config == "drop"
    # the contact drop: mu = 0.5 on the ground and the box, and a sideways start (0.3, 0.1) m/s next to the
    # 1 m/s fall so that contacts both slide and stick
    sc = (scenes.drop_blob(res=args.drop_res, friction=args.friction,
                           lateral=(0.3, 0.1) if args.friction > 0 else (0.0, 0.0))
          if drop else scenes.config(args.config))
    if args.energy >= 0:
        sc = dataclasses.replace(sc, energy=args.energy, name=f"{sc.name}_energy{args.energy}")
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")  # noqa: E731
    # adjoint: start extrapolated (quadratically) from the sweep's previous solutions (runs to ADJ_TOL either way)
    g = Scene.from_scene(sc, eps_adj=ADJ_TOL, max_sub=args.max_sub, adj_warm=3, iface_levels=args.iface_levels)
    info = g.info()
    print(f"[bench] scene {sc.name}: {info}", file=sys.stderr, flush=True)
    # warmup (untimed)
    if args.warmup > 0:
        rollout_fwd_bwd(g, sc, args.warmup, torch, dev)
        print("[bench] warmup done", file=sys.stderr, flush=True)
    # timed region, with per-launch HIP-event timing of one kernel on the
    # library's stream
    kid = KERNELS[args.timed_kernel]
    g.kernel_timer(kid)
    dt, fiters, biters, g_logE = rollout_fwd_bwd(g, sc, args.steps, torch, dev)
    ktime_ms, kcount, kwork = g.kernel_timer_read()
    g.kernel_timer(-1)
    assert torch.isfinite(g_logE).all()
    print(f"[bench] timed {args.steps} fwd+bwd steps in {dt:.4f} s; fwd iters/step {np.mean(fiters):.2f}, "
          f"adjoint iters/step {np.mean(biters):.2f}", file=sys.stderr, flush=True)
    if drop:
        print(f"[bench] contact rows/step {np.mean(g.contact_hist):.1f}, max {max(g.contact_hist)}; active max "
              f"{max(g.active_hist)}", file=sys.stderr, flush=True)
    value = args.steps / dt
    # roofline of the timed kernel: algorithmic bytes of the units that did
    # work over the summed launch durations
    bytes_per_unit = g.kernel_bytes(kid)
    traffic = measured_traffic(args.timed_kernel, args.config, args.drop_res)
    roof = roofline_entry(args.timed_kernel, "hbm", ktime_ms, kcount, kwork * bytes_per_unit, HBM_PEAK_GBS, "GB/s",
                          traffic=traffic, extra={"working_units": int(kwork),
                                                  "algorithmic_bytes_per_unit": int(bytes_per_unit),
                                                  "nnz_L": round(g.factor_nnz())})
    out = {"metric": METRIC, "value": round(value, 3), "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(1000.0 * dt / args.steps, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": (f"{sc.name}: voxelised blob of 6 spheres, {sc.n_e} tets, {sc.n_v} verts, shell "
                                   f"E 1e6 over interior 1e4, nu 0.49, h {sc.h}, dropped at 1 m/s onto the ground "
                                   f"plane and a box"
                                   + (f" with a sideways start of (0.3, 0.1) m/s, Coulomb friction mu "
                                      f"{sc.friction:g} (one frame of three rows per contact vertex), "
                                      f"projected fixed-point adjoint through the frictional rows to {ADJ_TOL:g}"
                                      if sc.friction > 0 else
                                      f", frictionless contact, adjoint PCG to {ADJ_TOL:g}")
                                   + f", rollout of {args.steps} steps, gate 1e-6, FB residual 1e-10") if drop else
                                  (f"{sc.name}: 40x10x10 cubes, {sc.n_e} tets, {sc.n_v} verts, "
                                   + ("homogeneous E 1e5, nu 0.45, 16 muscle groups (4 segments x 4 quadrants) with "
                                      "fibres on a 30 degree helix, seeded activations in [0, 0.3], gravity"
                                      if sc.muscle_group is not None else
                                      "two-phase E 1e4/1e6, nu 0.49")
                                   + (["", ", corotated + volume composite energy",
                                       ", logarithmic volume-barrier energy"][sc.energy])
                                   + f", h {sc.h}, rollout of {args.steps} steps, AA window {sc.aa_window}, "
                                   f"gate 1e-6, adjoint PCG to {ADJ_TOL:g}, plain q0 = q_t, adjoint start "
                                   "extrapolated from the last three solutions"),
                      "fwd_iters_per_step": round(float(np.mean(fiters)), 3),
                      "adj_iters_per_step": round(float(np.mean(biters)), 3),
                      "n_subdomains": int(info["n_subdomains"]), "n_interface": int(info["n_interface"])},
           "roofline": roof}
    if drop:
        out["config"]["contact_rows_per_step"] = round(float(np.mean(g.contact_hist)), 2)
        out["config"]["max_active_rows"] = int(max(g.active_hist))
    if not args.no_warm_run:
        out["warm_started"] = {}
        # the same rollout with the inertial first iterate q0 = q_t + h v_t
        gw = Scene.from_scene(sc, eps_adj=ADJ_TOL, max_sub=args.max_sub, adj_warm=3, fwd_start=1,
                              iface_levels=args.iface_levels)
        if args.warmup > 0:
            rollout_fwd_bwd(gw, sc, args.warmup, torch, dev)
        dtw, fw, bw, _ = rollout_fwd_bwd(gw, sc, args.steps, torch, dev)
        out["warm_started"]["inertial"] = {"value": round(args.steps / dtw, 3), "unit": "steps/s",
                                           "ms_per_step": round(1000.0 * dtw / args.steps, 4),
                                           "fwd_iters_per_step": round(float(np.mean(fw)), 3),
                                           "adj_iters_per_step": round(float(np.mean(bw)), 3),
                                           "start": "q0 = q_t + h v_t"}
        print(f"[bench] inertial start: {args.steps / dtw:.1f} steps/s", file=sys.stderr, flush=True)
        # the learned start: a network trained here, on the GPU, on plain rollouts of other members of the
        # scene's family (other beams; drops of the same blob with other initial velocities)
        from paper_2605_14526_amd import warmstart
        if drop:
            fam = lambda k: scenes.drop_family(k, res=args.drop_res, steps=100, friction=args.friction)  # noqa: E731
        else:
            fam = lambda k: scenes.hetero_beam_family(k, steps=args.steps)  # noqa: E731
        net, hist, tsec, nsamp = warmstart.train_for(fam, args.train_scenes, 100, args.train_epochs, torch, seed=1,
                                                     edge_weight=LEARNED_EDGE_WEIGHT)
        logw = torch.tensor(g.vertex_logw(), dtype=torch.float64, device="cuda")
        if args.warmup > 0:
            rollout_fwd_bwd(g, sc, args.warmup, torch, dev, net, logw)
        dtl, fl, bl, _ = rollout_fwd_bwd(g, sc, args.steps, torch, dev, net, logw)
        out["warm_started"]["learned"] = {"value": round(args.steps / dtl, 3), "unit": "steps/s",
                                          "ms_per_step": round(1000.0 * dtl / args.steps, 4),
                                          "fwd_iters_per_step": round(float(np.mean(fl)), 3),
                                          "adj_iters_per_step": round(float(np.mean(bl)), 3),
                                          "start": "message-passing network (BF16 matrix cores), inference timed, "
                                                   "trained on " + ("drops of the same blob with other initial "
                                                                    "velocities" if drop else "other beams"),
                                          "train": {"scenes": args.train_scenes, "samples": nsamp,
                                                    "epochs": args.train_epochs, "seconds": round(tsec, 2),
                                                    "final_loss": hist[-1]}}
        print(f"[bench] learned start: {args.steps / dtl:.1f} steps/s, fwd iters/step {np.mean(fl):.2f} "
              f"(trained {tsec:.1f} s)", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        n = args.cpu_sample_steps
        if sc.tets.shape[0] > 50000:  # the oracle's reverse sweep takes seconds per step at this size
            n = 1
        out["cpu_baseline"] = cpu_baseline_entry([(sc, n)], [(sc, min(n, 2))],
                                                 f"first {n} fwd+bwd steps of the same rollout")
        out["cpu_baseline"]["unit"] = "steps/s"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
