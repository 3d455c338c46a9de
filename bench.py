"""Benchmark of the fused phase-field lattice Boltzmann step on one MI355X.

Workload: D3Q19 rising bubble, 128^3 sites, periodic in x and y, walls in z,
rho_H/rho_L = 1000, mu_H/mu_L = 100, R = 16, W = 4, Eotvos number 10, hydrostatic
start; distributions stored in FP32 (the value), with FP16-shifted storage timed beside
it (speed-up and the phi difference between the two after the same steps).  Further
blocks: the D3Q19 droplet impact on a film (256x256x128) and the same rising bubble on
256^3, both storages; the D2Q9 Rayleigh-Taylor case (256x1024); the top wall moving;
contact angles of 60 and 120 degrees on the bottom and top walls; the largest domain the
library accepts (1000x1000x268 sites);
and the learned 16-step surrogate (D2Q9 256^2 droplets): trained here on solver
trajectories, then its held-out error, its forward/training rate against the BF16 MFMA
peak, and its speed against 16 plain steps (batched over the domains) with the guard.

A step is one fused stream-and-collide pass over both distribution sets (every site,
every population); the sum(phi)/non-finite guard runs once at the end of the timed
region.  Inputs are resident in HBM before timing starts.  The value is million
lattice-site updates per second (MLUPS) of the whole GPU.

Prints one JSON line.
"""
import hashlib
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D3Q19 two-set MLUPS & % HBM roofline; FP16-store/surrogate vs FP32 at stated φ err"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per site update: read + write of both sets once (FP16S: per site
# the float32 rest populations of both sets and an fp16 moments word of 8 values, and
# per moving population one fp16 deviation per set)
BYTES_PER_SITE = {("19", "fp32"): 2 * 2 * 19 * 4, ("19", "fp16s"): 2 * (8 + 16 + 18 * 4),
                  ("9", "fp32"): 2 * 2 * 9 * 4, ("9", "fp16s"): 2 * (8 + 16 + 8 * 4),
                  # in place: the phi pass reads the Q h values and writes phi, the step
                  # reads phi and both sets and writes both sets
                  ("19", "fp32_inplace"): 19 * 4 + 4 + 4 + 2 * 2 * 19 * 4,
                  ("9", "fp32_inplace"): 9 * 4 + 4 + 4 + 2 * 2 * 9 * 4}
# device bytes of the state per site (both buffers of the pull storages, one in place)
STATE_BYTES = {"fp32": 2 * 19 * 8, "fp16s": 2 * (8 + 16 + 18 * 4), "fp32_inplace": 19 * 8}
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "k_step_rising_bubble_traffic.txt")
CSRC = os.path.join(ROOT, "paper_1812_00118_amd", "csrc")


STEP_SOURCES = ("pflb_device.hpp", "pflb_internal.hpp", "pflb_kernels.hip")


def kernel_source_sha1():
    """Hash of the step kernel's sources: counter figures taken for another build of it
    are not used."""
    h = hashlib.sha1()
    for f in STEP_SOURCES:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()[:16]


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--storage", choices=["fp16s", "fp32", "fp32_inplace"], default="fp32",
                    help="fp32_inplace only with --no-compare (kernel traces of that storage)")
    ap.add_argument("--workload", choices=["rising_bubble", "droplet_impact"],
                    default="rising_bubble")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the other storage mode and the CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--sur-train-steps", type=int, default=6000)
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--sur-profile", action="store_true",
                    help="only run 3 surrogate forward passes at batch 32 and 2 training steps "
                         "at batch 8 (random weights; for a kernel trace)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 4 plain device copies of MIB MiB (counter calibration)")
    return ap.parse_args()


def copy_probe(mib):
    """Four device-to-device copies of a known size: FETCH_SIZE and WRITE_SIZE of these
    dispatches calibrate the HBM counters (each should read mib MiB)."""
    import torch
    n = mib * 1024 * 1024 // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(4):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 4, "copies": 4}), flush=True)


def copy_ceiling(moved_bytes, reps=20):
    """GB/s of a device-to-device copy that reads and writes moved_bytes / 2 each: the
    rate a kernel moving the same bytes (read once, written once) could reach at best on
    this GPU."""
    import torch
    n = moved_bytes // 2 // 4
    src = torch.ones(n, device="cuda")
    dst = torch.empty_like(src)
    ms = _events_ms(lambda: dst.copy_(src), reps)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * n * 4 / (ms * 1e-3) / 1e9


def time_storage(cfg, storage, steps, warmup, perturb_seed=None):
    """Time `steps` steps after `warmup`; perturb_seed: start from phi moved by float32
    half-ulp noise (relative 2^-24, seeded), for the conditioning of the run."""
    import numpy as np
    import torch
    from paper_1812_00118_amd import Sim
    import pfinputs
    phi, u, P = pfinputs.fields(cfg)
    if perturb_seed is not None:
        rng = np.random.default_rng(perturb_seed)
        phi = (phi.astype(np.float64) *
               (1.0 + 2.0 ** -24 * rng.standard_normal(phi.shape))).astype(np.float32)
    sim = Sim(cfg, storage=storage)
    sim.init_fields(phi, u, P)
    sim.release_work()
    sim.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    mass, bad = sim.mass()           # guard: synchronous, ends the timed region
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = e0.elapsed_time(e1) / steps
    phi_out = sim.read(fields=("phi",))["phi"]
    return dict(kernel_ms=kernel_ms, wall_s=wall, mass=mass, nonfinite=bad, phi=phi_out,
                steps_done=sim.steps)


def time_graph(cfg, storage, steps, warmup):
    """Kernel time per step when the steps are replayed from one captured HIP graph
    (pflb_step_graph) on a created stream."""
    import torch
    from paper_1812_00118_amd import Sim
    import pfinputs
    sim = Sim(cfg, storage=storage)
    sim.init_fields(*pfinputs.fields(cfg))
    sim.release_work()
    sim.step(warmup)
    torch.cuda.synchronize()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        sim.step_graph(steps)            # capture and first replay
        st.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        sim.step_graph(steps)
        e1.record(st)
        st.synchronize()
    return e0.elapsed_time(e1) / steps


def largest_domain_block(steps=20, warmup=5):
    """The step on the largest domain that fits the device's free memory, per storage:
    1000 x 1000 x nz sites of the rising-bubble fluid with a bubble of radius 64, its phi
    built on the device (u = 0, P = 0).  Beyond 2^28 - 64 sites the kernels address the
    slots with 64-bit sums."""
    import torch
    from paper_1812_00118_amd import Sim
    import pfinputs
    nx, ny, R = 1000, 1000, 64.0
    blk = {"workload": "rising_bubble D3Q19 1000 x 1000 x nz, the largest nz the free device "
                       "memory holds (state, the start's work buffer and fields), x,y "
                       "periodic, z walls, R 64"}
    dev = torch.device("cuda")
    for st in ("fp32", "fp16s", "fp32_inplace"):
        # the state, the 2 Q N floats of the start's work (none in place, where the
        # equilibria go straight into the state; the phi field instead), phi and u
        # (16 B), and the temporaries of building phi
        per_site = STATE_BYTES[st] + (4 if st == "fp32_inplace" else 2 * 19 * 4) + 16 + 24
        free = torch.cuda.mem_get_info()[0]
        nz = int(0.92 * free / per_site / (nx * ny))
        nz = min(nz, (2 ** 32 - 64) // (nx * ny))
        if nz < 8:
            blk[st] = {"skipped": "not enough free device memory"}
            continue
        n = nx * ny * nz
        cfg = dict(pfinputs.rising_bubble(R=R), shape=(nx, ny, nz))
        z = torch.arange(nz, device=dev, dtype=torch.float32).view(nz, 1, 1)
        y = torch.arange(ny, device=dev, dtype=torch.float32).view(1, ny, 1)
        x = torch.arange(nx, device=dev, dtype=torch.float32).view(1, 1, nx)
        r = torch.sqrt((x - (nx - 1) / 2) ** 2 + (y - (ny - 1) / 2) ** 2 + (z - 2 * R) ** 2)
        phi = 0.5 + 0.5 * torch.tanh(2.0 * (r - R) / cfg["W"])
        del x, y, z, r
        u = torch.zeros((3, nz, ny, nx), device=dev)
        sim = Sim(cfg, storage=st)
        sim.init_fields(phi, u)
        del phi, u
        sim.release_work()
        torch.cuda.empty_cache()
        sim.step(warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        sim.step(steps)
        e1.record()
        _, bad = sim.mass()
        ms = e0.elapsed_time(e1) / steps
        blk[st] = {"shape": [nx, ny, nz], "sites": n, "addr64": n > 2 ** 28 - 64,
                   "state_GB": round(STATE_BYTES[st] * n / 1e9, 1),
                   "mlups": round(n / (ms * 1e-3) / 1e6, 1), "kernel_ms": round(ms, 3),
                   "achieved_GBs": round(BYTES_PER_SITE[("19", st)] * n / (ms * 1e-3) / 1e9, 1),
                   "nonfinite": bad}
        print(f"[bench] largest domain {st}: {nx}x{ny}x{nz} ({n:.3g} sites), {ms:.3f} ms/step",
              file=sys.stderr, flush=True)
        del sim
        torch.cuda.empty_cache()
    return blk


def read_traffic(storage):
    """HBM bytes per launch from the committed rocprofv3 counter summary (null if the
    summary is absent or was taken for another kernel build)."""
    try:
        lines = open(PROFILE_TRAFFIC).read().splitlines()
    except OSError:
        return None
    vals = {}
    for ln in lines:
        if "=" in ln:
            k, v = ln.split("=", 1)
            vals[k.strip()] = v.strip().split()[0] if v.strip() else ""
    if vals.get("source_sha1") != kernel_source_sha1():
        return None
    v = vals.get(f"traffic_bytes_per_launch[{storage}]")
    return float(v) if v else None


def _oracle_rate(n, R, seconds, min_steps=2):
    """Whole-domain FP64 oracle steps of the rising bubble on n^3 sites (same fluid
    parameters, bubble radius R) for about `seconds`: (sites, steps, elapsed)."""
    import numpy as np
    import pfinputs
    from oracle import pflbm as O
    cfg = pfinputs.rising_bubble(n=n, R=R)
    prm = O.Params.from_dict(pfinputs.model_params(cfg))
    phi, u, P = pfinputs.fields(cfg)
    h, g = O.init(prm, phi.astype(np.float64), u.astype(np.float64), P.astype(np.float64))
    h, g = O.step(prm, h, g)            # warm-up
    k, t0 = 0, time.perf_counter()
    while True:
        h, g = O.step(prm, h, g)
        k += 1
        el = time.perf_counter() - t0
        if el >= seconds and k >= min_steps:
            break
    return n ** 3, k, el


def _oracle_worker(args):
    n, R, seconds = args
    return _oracle_rate(n, R, seconds)


def cpu_baseline(seconds):
    """The FP64 oracle timed on the host, before the GPU is touched.
    All cores: one oracle process per core, each stepping a 48^3 sub-box of the rising
    bubble (same fluid parameters, bubble scaled to R = 6); the value is their summed
    rate.  One core: the oracle stepping the full 128^3 rising bubble (the benchmark's
    own workload) for a few whole-domain steps."""
    import multiprocessing as mp
    cores = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                       else (os.cpu_count() or 1)))
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_worker, [(48, 6.0, seconds)] * cores)
    agg = sum(s * k / el for s, k, el in res) / 1e6
    out = {"value": round(agg, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
           "sample": f"{cores} oracle processes (numpy, one thread each) side by side, each "
                     f"stepping a 48^3 sub-box of the rising bubble (R 6, same fluid "
                     f"parameters) for ~{seconds:.0f} s; value = summed sites x steps / s"}
    sites, k, el = _oracle_rate(128, 16.0, seconds, min_steps=1)
    out["single_core"] = {"mlups": round(sites * k / el / 1e6, 3), "steps": k,
                          "seconds": round(el, 2),
                          "sample": "the full 128^3 rising bubble, numpy single thread"}
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")),
                         "")
    except OSError:
        pass
    out["host"] = {"cpu_model": model, "logical_cpus": os.cpu_count(), "cores_used": cores}
    return out


def _sur_input(shape, seed):
    """Seeded standard-normal network inputs for the timing runs: the kernels' speed
    depends on the data on this GPU (all-zero inputs run about 10% faster), so the timed
    forward passes see values that exercise every bit."""
    import torch
    g = torch.Generator(device="cuda").manual_seed(seed)
    return torch.randn(shape, generator=g, device="cuda")


def _events_ms(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / reps


def surrogate_block(train_steps):
    """Train the surrogate on solver trajectories (D2Q9 256^2 droplets), then measure
    its held-out error and its speed against the plain solver."""
    import numpy as np
    import torch
    import pfinputs
    from paper_1812_00118_amd import Sim, surrogate as S, sur_train as T

    H = W = 256
    t0 = time.time()
    tr = T.Dataset(range(128), pfinputs.drops, t0=64, n_states=9)
    te = T.Dataset(range(2000, 2004), pfinputs.drops, t0=64, n_states=9)
    gen_s = time.time() - t0
    norm = T.normalisation(tr)
    sur = S.Surrogate(H, W, 32, norm)
    sur.set_params(S.init_params(0))
    t0 = time.time()
    losses = T.train(sur, tr, train_steps, 16, 1e-3, seed=0)
    torch.cuda.synchronize()
    train_s = time.time() - t0
    ev = T.evaluate(sur, te)
    print(f"[bench] surrogate: trained {train_steps} steps in {train_s:.1f} s; test mse "
          f"{ev['mse']:.4f} (persistence {ev['mse_persistence']:.4f}), phi err "
          f"{ev['phi_err']:.4f} (persistence {ev['phi_err_persistence']:.4f})",
          file=sys.stderr, flush=True)
    flops = sum(2 * H * W // 4 ** lvl * cout * 9 * cin for (_, cin, cout), lvl in
                zip(S.LAYERS, [0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 2, 1, 1, 1, 0, 0, 0]))
    flops += 2 * H * W * S.HEAD[0] * S.HEAD[1]
    fwd = {}
    for B in (1, 32):
        x = _sur_input((B, H, W, S.IN_CH), 1).to(torch.bfloat16)
        fwd[B] = _events_ms(lambda: sur.forward(x), 20 if B == 1 else 10)
    xb = _sur_input((8, H, W, S.IN_CH), 2).to(torch.bfloat16)
    yb = _sur_input((8, H, W, S.OUT_CH), 3)
    train_ms = _events_ms(lambda: sur.train_step(xb, yb, 0.0), 4)
    # plain solver: 16 steps of one 256^2 domain
    cfg = pfinputs.drops(2000)
    sim = Sim(pfinputs.model_params(cfg))
    sim.init_fields(*pfinputs.fields(cfg))
    sim.release_work()
    lb16 = _events_ms(lambda: sim.step(16), 20)
    # the same for 32 domains, batched (one launch per step for every 16 domains)
    sims32 = []
    for k in range(32):
        c32 = pfinputs.drops(2000 + k)
        sm = Sim(pfinputs.model_params(c32))
        sm.init_fields(*pfinputs.fields(c32))
        sm.release_work()
        sims32.append(sm)
    lb16_b32 = _events_ms(lambda: Sim.step_many(sims32, 16), 10)
    del sims32
    # guarded advance vs plain steps from the same states: 8 windows (128 steps), every
    # 4th window checked against the plain steps; one context, and a batch of 32
    guarded = {}
    for nb in (1, 32):
        seeds = list(range(2000, 2000 + nb))
        cfgs = [pfinputs.drops(k) for k in seeds]
        a, b, c1 = [], [], []
        for c in cfgs:
            for lst in (a, b, c1):
                sm = Sim(pfinputs.model_params(c))
                sm.init_fields(*pfinputs.fields(c))
                sm.release_work()
                sm.step(64)
                lst.append(sm)
        torch.cuda.synchronize()
        m_start = [sm.mass()[0] for sm in a]
        t0 = time.time()
        nf = sur.advance_guarded(a, 8, mass_tol=1e-3, phi_tol=0.05, check_every=4,
                                 u_max=0.1)
        torch.cuda.synchronize()
        g_ms = (time.time() - t0) * 1e3
        drift = max(abs(sm.mass()[0] - m0) / m0 for sm, m0 in zip(a, m_start))
        # plain stepping, batched (the fair baseline), and one domain after another
        t0 = time.time()
        Sim.step_many(b, 128)
        torch.cuda.synchronize()
        p_ms = (time.time() - t0) * 1e3
        t0 = time.time()
        for sm in c1:
            sm.step(128)
        torch.cuda.synchronize()
        p1_ms = (time.time() - t0) * 1e3
        for x, y in zip(b, c1):
            assert torch.equal(x.read(("phi",))["phi"], y.read(("phi",))["phi"])
        # phi error after 128 steps against the plain solver: the max-norm is set by the
        # worst interface (a sub-site shift of a steep profile), so the mean and the share
        # of sites off by more than 0.1 are reported beside it
        diffs = torch.stack([(x.read(("phi",))["phi"] - y.read(("phi",))["phi"]).abs()
                             for x, y in zip(a, b)])
        dphi = diffs.max().item()
        mphi = diffs.mean().item()
        frac = (diffs > 0.1).float().mean().item()
        guarded[f"batch{nb}"] = {"contexts": nb, "windows": 8, "check_every": 4, "u_max": 0.1,
                                 "fallbacks": nf, "fallback_rate": round(nf / (8 * nb), 4),
                                 "wall_ms": round(g_ms, 3), "plain_lb_ms": round(p_ms, 3),
                                 "speedup": round(p_ms / g_ms, 3),
                                 "plain_lb_ms_one_domain_at_a_time": round(p1_ms, 3),
                                 "max_abs_dphi_vs_lb_after_128_steps": dphi,
                                 "mean_abs_dphi_vs_lb_after_128_steps": mphi,
                                 "share_of_sites_abs_dphi_over_0.1": frac,
                                 "max_rel_sum_phi_drift_over_128_steps": drift}
        print(f"[bench] guarded batch {nb}: {g_ms:.1f} ms vs plain {p_ms:.1f} ms batched "
              f"({p1_ms:.1f} ms one domain at a time), fallbacks "
              f"{nf}/{8 * nb}, max|dphi| {dphi:.3e}, mean|dphi| {mphi:.2e}, "
              f"sites |dphi|>0.1 {frac:.2e}", file=sys.stderr, flush=True)
        del a, b, c1
    ach = flops * 32 / (fwd[32] * 1e-3) / 1e12
    return {
        "workload": "drops D2Q9 256^2 periodic, 2-8 droplets, R U[8,32], rho_H logU[10,1000]",
        "params": int(sur.nparams),
        "gflop_per_sample_forward": round(flops / 1e9, 3),
        "train": {"pairs": len(tr), "trajectories": 128, "steps": train_steps, "batch": 16,
                  "seconds": round(train_s, 2), "data_seconds": round(gen_s, 2),
                  "final_loss": round(float(np.mean(losses[-20:])), 5)},
        "test": {k: round(v, 5) for k, v in ev.items()},
        "forward_ms": {"batch1": round(fwd[1], 4), "batch32": round(fwd[32], 4)},
        "train_step_ms_batch8": round(train_ms, 4),
        "lb16_ms_per_domain": round(lb16, 4),
        "lb16_ms_32_domains_batched": round(lb16_b32, 4),
        "speedup_vs_lb16": {"batch1": round(lb16 / fwd[1], 4),
                            "batch32": round(lb16_b32 / fwd[32], 4)},
        "roofline": {"bound": "mfma", "achieved": round(ach, 2), "peak": 2500.0,
                     "unit": "TFLOP/s", "frac": round(ach / 2500.0, 5),
                     "kernel": "forward, batch 32 (17 conv + head)"},
        "guarded": dict(guarded, mass_tol=1e-3, phi_tol=0.05),
    }


def sur_profile():
    import torch
    from paper_1812_00118_amd import surrogate as S
    norm = dict(in_shift=[0.0] * 4, in_scale=[1.0] * 4, out_scale=[1.0] * 4, lrr_scale=1.0)
    sur = S.Surrogate(256, 256, 32, norm)
    sur.set_params(S.init_params(0))
    x = _sur_input((32, 256, 256, S.IN_CH), 1).to(torch.bfloat16)
    fwd = [_events_ms(lambda: sur.forward(x), 1) for _ in range(3)]
    xb = _sur_input((8, 256, 256, S.IN_CH), 2).to(torch.bfloat16)
    yb = _sur_input((8, 256, 256, S.OUT_CH), 3)
    trn = _events_ms(lambda: sur.train_step(xb, yb, 0.0), 2)
    print(json.dumps({"forward_ms_batch32": round(min(fwd), 4),
                      "train_step_ms_batch8": round(trn, 4)}), flush=True)


def main():
    args = parse_args()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.sur_profile:
        sur_profile()
        return
    if args.storage == "fp32_inplace" and not args.no_compare:
        print("--storage fp32_inplace needs --no-compare (the full run reports the in-place "
              "storage in its own block)", file=sys.stderr)
        sys.exit(2)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU slab "
              f"decomposition is a design note, not part of this build.", file=sys.stderr)
        sys.exit(2)
    cpu = None
    if not args.no_compare:
        # the oracle's worker processes are forked before this process touches the GPU
        t0 = time.time()
        cpu = cpu_baseline(args.cpu_seconds)
        print(f"[bench] cpu baseline: {cpu['value']} MLUPS on {cpu['cores']} cores, "
              f"{cpu['single_core']['mlups']} MLUPS one core ({time.time() - t0:.0f} s)",
              file=sys.stderr, flush=True)
    import torch
    import pfinputs
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    cfg = pfinputs.rising_bubble() if args.workload == "rising_bubble" else pfinputs.droplet_impact()
    nx, ny, nz = cfg["shape"]
    N = nx * ny * nz
    desc = {"rising_bubble": "rising_bubble D3Q19 128^3 (x,y periodic, z walls, rho 1000, "
                             "mu 100, R 16, W 4, Eo 10, hydrostatic start)",
            "droplet_impact": "droplet_impact D3Q19 256x256x128 (x,y periodic, z walls, "
                              "rho 1000, R 32, film 16, U 0.05, Re 500, We 8000)"}
    print(f"[bench] workload {args.workload} {nx}x{ny}x{nz}, storage {args.storage}, "
          f"warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
    main_run = time_storage(cfg, args.storage, args.steps, args.warmup)
    ms = main_run["kernel_ms"]
    mlups = N / (ms * 1e-3) / 1e6
    bps = BYTES_PER_SITE[("19", args.storage)]
    achieved = bps * N / (ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_run["wall_s"] * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc[args.workload], "storage": args.storage, "sites": N},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": read_traffic(args.storage),
                     "kernel": ("k_ip_phi + k_ip_step<D3Q19>" if args.storage == "fp32_inplace"
                                else "k_step<D3Q19>"), "bytes_per_site": bps,
                     "kernel_ms": round(ms, 4)},
        "nonfinite": main_run["nonfinite"],
    }
    # the same bytes moved by a plain device-to-device copy on this GPU (context for the
    # fraction of the 8 TB/s peak: a copy does not reach it either)
    copy_gbs = copy_ceiling(bps * N)
    out["roofline"]["copy_GBs"] = round(copy_gbs, 1)
    out["roofline"]["frac_of_copy"] = round(achieved / copy_gbs, 4)
    print(f"[bench] {args.storage}: {ms:.4f} ms/step, {mlups:.0f} MLUPS, "
          f"{achieved:.0f} GB/s", file=sys.stderr, flush=True)
    if not args.no_compare:
        other = "fp32" if args.storage == "fp16s" else "fp16s"
        o = time_storage(cfg, other, args.steps, args.warmup)
        oms = o["kernel_ms"]
        dphi = (main_run["phi"] - o["phi"]).abs().max().item()
        out["compare"] = {
            "storage": other,
            "mlups": round(N / (oms * 1e-3) / 1e6, 1),
            "kernel_ms": round(oms, 4),
            "achieved_GBs": round(BYTES_PER_SITE[("19", other)] * N / (oms * 1e-3) / 1e9, 1),
            "speedup_fp16s_vs_fp32": round((ms / oms) if other == "fp16s" else (oms / ms), 3),
            "max_abs_dphi_fp16s_vs_fp32": dphi,
            "after_steps": main_run["steps_done"],
        }
        # the run's own conditioning: FP32 against FP32 from a start whose phi moved by
        # float32 half-ulp noise, after the same steps
        fp32_run = main_run if args.storage == "fp32" else o
        p = time_storage(cfg, "fp32", args.steps, args.warmup, perturb_seed=7)
        cond = (p["phi"] - fp32_run["phi"]).abs().max().item()
        out["compare"]["max_abs_dphi_fp32_vs_fp32_halfulp_start"] = cond
        print(f"[bench] {other}: {oms:.4f} ms/step; max|dphi| fp16s vs fp32 {dphi:.2e} "
              f"(fp32 vs fp32 from a half-ulp start: {cond:.2e})", file=sys.stderr, flush=True)
        if args.workload == "rising_bubble":
            cfg2 = pfinputs.droplet_impact()
            n2 = 256 * 256 * 128
            blk = {"workload": desc["droplet_impact"]}
            for st in ("fp32", "fp16s"):
                r2 = time_storage(cfg2, st, max(50, args.steps // 4), args.warmup)
                blk[st] = {"mlups": round(n2 / (r2["kernel_ms"] * 1e-3) / 1e6, 1),
                           "kernel_ms": round(r2["kernel_ms"], 4),
                           "achieved_GBs": round(BYTES_PER_SITE[("19", st)] * n2 /
                                                 (r2["kernel_ms"] * 1e-3) / 1e9, 1)}
                print(f"[bench] droplet_impact {st}: {r2['kernel_ms']:.4f} ms/step",
                      file=sys.stderr, flush=True)
            out["droplet_impact"] = blk
            # the same rising bubble on 256^3 (16.8 M sites, 5.1 GB of FP32 state)
            cfg5 = pfinputs.rising_bubble(n=256, R=32.0)
            n5 = 256 ** 3
            blk = {"workload": "rising_bubble D3Q19 256^3 (x,y periodic, z walls, R 32, "
                               "otherwise as the 128^3 case)"}
            for st in ("fp32", "fp16s"):
                r5 = time_storage(cfg5, st, max(20, args.steps // 20), args.warmup)
                blk[st] = {"mlups": round(n5 / (r5["kernel_ms"] * 1e-3) / 1e6, 1),
                           "kernel_ms": round(r5["kernel_ms"], 4),
                           "achieved_GBs": round(BYTES_PER_SITE[("19", st)] * n5 /
                                                 (r5["kernel_ms"] * 1e-3) / 1e9, 1)}
                print(f"[bench] rising_bubble 256^3 {st}: {r5['kernel_ms']:.4f} ms/step",
                      file=sys.stderr, flush=True)
            blk["speedup_fp16s_vs_fp32"] = round(blk["fp32"]["kernel_ms"] /
                                                 blk["fp16s"]["kernel_ms"], 3)
            out["rising_bubble_256"] = blk
            # D2Q9 Rayleigh-Taylor (256 x 1024, y walls): 38 MB of state per set, so the
            # step runs largely from the 256 MB Infinity Cache; reported as effective rates
            cfg3 = pfinputs.rayleigh_taylor()
            n3 = 256 * 1024
            blk = {"workload": "rayleigh_taylor D2Q9 256x1024 (x periodic, y walls, Atwood 0.5, "
                               "g 1e-5, W 5, Re 3000)"}
            for st in ("fp32", "fp16s"):
                r3 = time_storage(cfg3, st, max(200, args.steps), args.warmup)
                blk[st] = {"mlups": round(n3 / (r3["kernel_ms"] * 1e-3) / 1e6, 1),
                           "kernel_ms": round(r3["kernel_ms"], 5),
                           "effective_GBs": round(BYTES_PER_SITE[("9", st)] * n3 /
                                                  (r3["kernel_ms"] * 1e-3) / 1e9, 1)}
                gms = time_graph(cfg3, st, max(200, args.steps), args.warmup)
                blk[st]["graph_kernel_ms"] = round(gms, 5)
                print(f"[bench] rayleigh_taylor {st}: {r3['kernel_ms']:.4f} ms/step "
                      f"({gms:.4f} replayed from a HIP graph)", file=sys.stderr, flush=True)
            blk["graph"] = ("graph_kernel_ms: the same steps captured once with "
                            "pflb_step_graph and replayed as one graph launch")
            out["rayleigh_taylor"] = blk
            # moving walls: the rising-bubble domain with its top wall sliding along x
            # (the step variant with momentum-corrected bounce-back)
            cfg4 = dict(cfg, wall_u=[[0.0] * 3] * 5 + [[0.01, 0.0, 0.0]])
            blk = {"workload": "rising_bubble D3Q19 128^3, z+ wall moving at 0.01 along x"}
            for st in ("fp32", "fp16s"):
                r4 = time_storage(cfg4, st, max(50, args.steps // 4), args.warmup)
                rest = ms if st == args.storage else oms
                blk[st] = {"mlups": round(N / (r4["kernel_ms"] * 1e-3) / 1e6, 1),
                           "kernel_ms": round(r4["kernel_ms"], 4),
                           "achieved_GBs": round(BYTES_PER_SITE[("19", st)] * N /
                                                 (r4["kernel_ms"] * 1e-3) / 1e9, 1),
                           "time_vs_resting_walls": round(r4["kernel_ms"] / rest, 3)}
                print(f"[bench] moving_walls {st}: {r4['kernel_ms']:.4f} ms/step "
                      f"({r4['kernel_ms'] / rest:.3f}x the resting-wall step)",
                      file=sys.stderr, flush=True)
            out["moving_walls"] = blk
            try:
                out["largest_domain"] = largest_domain_block()
            except torch.cuda.OutOfMemoryError:
                import gc
                gc.collect()
                torch.cuda.empty_cache()
                out["largest_domain"] = {"skipped": "out of device memory"}
            # contact angles: the rising-bubble domain with 60 degrees on the bottom and
            # 120 on the top wall (the step variant with the wetting ghost rule)
            cfg5 = dict(cfg, wet_cos=[0.0] * 4 + [0.5, -0.5])
            blk = {"workload": "rising_bubble D3Q19 128^3, contact angles 60 (z-) and 120 (z+) "
                               "degrees"}
            for st in ("fp32", "fp16s"):
                r5 = time_storage(cfg5, st, max(50, args.steps // 4), args.warmup)
                rest = ms if st == args.storage else oms
                blk[st] = {"mlups": round(N / (r5["kernel_ms"] * 1e-3) / 1e6, 1),
                           "kernel_ms": round(r5["kernel_ms"], 4),
                           "achieved_GBs": round(BYTES_PER_SITE[("19", st)] * N /
                                                 (r5["kernel_ms"] * 1e-3) / 1e9, 1),
                           "time_vs_90_degree_walls": round(r5["kernel_ms"] / rest, 3)}
                print(f"[bench] contact_angles {st}: {r5['kernel_ms']:.4f} ms/step "
                      f"({r5['kernel_ms'] / rest:.3f}x the 90-degree-wall step)",
                      file=sys.stderr, flush=True)
            out["contact_angles"] = blk
            # Section 4.4's dam break (its 537 x 198 x 50 box with the height along z):
            # the XBC step variant, which also stores the boundary layer's pressure,
            # and the open-face kernel after each step
            cfg6 = pfinputs.dam_break()
            n6 = 537 * 50 * 198
            blk = {"workload": "dam_break D3Q19 537x50x198 (the paper's 537x198x50, height "
                               "along z; no-slip walls, open top at P 0, water column H 100 "
                               "by 200, rho 1000, nu_water 4.9e-6, nu_air 8.3e-3, g 4e-6, "
                               "W 4, M 0.02, sigma 5.2e-3)"}
            for st in ("fp32", "fp16s"):
                r6 = time_storage(cfg6, st, max(50, args.steps // 4), args.warmup)
                blk[st] = {"mlups": round(n6 / (r6["kernel_ms"] * 1e-3) / 1e6, 1),
                           "kernel_ms": round(r6["kernel_ms"], 4),
                           "achieved_GBs": round(BYTES_PER_SITE[("19", st)] * n6 /
                                                 (r6["kernel_ms"] * 1e-3) / 1e9, 1),
                           "nonfinite": r6["nonfinite"]}
                print(f"[bench] dam_break {st}: {r6['kernel_ms']:.4f} ms/step",
                      file=sys.stderr, flush=True)
            out["dam_break"] = blk
            # in-place storage (one state buffer) on the headline workload
            blk = {"workload": desc[args.workload] + ", in-place FP32 storage",
                   "bytes_per_site": BYTES_PER_SITE[("19", "fp32_inplace")]}
            r7 = time_storage(cfg, "fp32_inplace", max(50, args.steps // 4), args.warmup)
            blk.update({"mlups": round(N / (r7["kernel_ms"] * 1e-3) / 1e6, 1),
                        "kernel_ms": round(r7["kernel_ms"], 4),
                        "achieved_GBs": round(BYTES_PER_SITE[("19", "fp32_inplace")] * N /
                                              (r7["kernel_ms"] * 1e-3) / 1e9, 1),
                        "time_vs_pull_fp32": round(r7["kernel_ms"] /
                                                   (ms if args.storage == "fp32" else oms), 3),
                        "nonfinite": r7["nonfinite"]})
            print(f"[bench] in-place fp32: {r7['kernel_ms']:.4f} ms/step",
                  file=sys.stderr, flush=True)
            out["inplace"] = blk
        if not args.no_surrogate:
            out["surrogate"] = surrogate_block(args.sur_train_steps)
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
