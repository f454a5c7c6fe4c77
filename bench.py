"""Benchmark: time-to-50-aperture plan on the prostate-shaped phantom (1 GPU).

One "step" is one whole plan: dao_solve from an empty pool to 50 apertures
(pricing, master, column generation) with the dose matrix resident on the
device.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--config prostate] [--cpu-seconds S]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# device sources of the master kernels; HBM traffic figures taken with
# rocprofv3 counters stay valid while these are unchanged
KERNEL_SOURCES = ["dao_common.h", "kernels.h", "kernels_ap.h", "kernels_coop.h"]
COPY_CALIB_BYTES = 512 << 20   # each of read and write of the calibration copy

METRIC = "time-to-50-aperture plan (s), plans/s + p50/p99; D·x, Dᵀg HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(ph, gpu_steps_per_plan, rounds_per_plan, seconds):
    """Time the FP64 oracle on the host on a bounded sample of the same plan.

    Sample: the oracle's own column generation on the same phantom, run
    round by round until `seconds` of CPU time are spent.  Its mean time per
    master step and per pricing round are scaled to one whole plan with the
    master step count the plan takes (the GPU runs the same algorithm).
    """
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    from oracle.master import MasterState, solve_master

    with threadpool_limits(limits=1):
        P = oracle.make_problem(ph.csr(), ph.rows_per_beam, ph.row_len, ph.vox_struct, ph.prescriptions)
        st = MasterState.empty(P)
        t_price = t_master = 0.0
        steps = rounds = 0
        rc1 = None
        t_all = time.perf_counter()
        while time.perf_counter() - t_all < seconds and rounds < ph.n_apertures:
            t0 = time.perf_counter()
            pr = oracle.price(P, st.g)
            t_price += time.perf_counter() - t0
            rc1 = rc1 if rc1 is not None else pr["rc"]
            st.add(pr["aperture"])
            t0 = time.perf_counter()
            budget = max(1, int(500))
            m = solve_master(P, st, tol=1e-6 * abs(rc1), max_steps=budget)
            t_master += time.perf_counter() - t0
            steps += m["steps"]
            rounds += 1
            if m["steps"] and (time.perf_counter() - t_all) > seconds:
                break
    s_step = t_master / max(1, steps)
    s_round = t_price / max(1, rounds)
    plan_s = s_step * gpu_steps_per_plan + s_round * rounds_per_plan
    return dict(value=1.0 / plan_s, unit="plans/s", cores=1, kind="oracle",
                sample=(f"FP64 oracle column generation on the same phantom for {rounds} rounds "
                        f"({steps} master steps, {t_master + t_price:.1f} s); {s_step * 1e3:.1f} ms per "
                        f"master step and {s_round * 1e3:.1f} ms per pricing round scaled to the "
                        f"{gpu_steps_per_plan} master steps and {rounds_per_plan} rounds of one plan"),
                plan_seconds=plan_s)


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1003_5402_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, config):
    """HBM bytes per launch of `kernel` from its committed counter summary
    (profiles/<kernel>_<config>_traffic.md: "key: value" lines), or None when
    there is none or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{config}_traffic.md")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip().strip("-* `")] = v.strip().strip("`")
    if kv.get("source_sha256") != kernel_source_hash():
        return None
    try:
        return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def pmc_workload(ctx, n_ap, torch):
    """Short run for counter collection: one plan, then a plain device copy
    of COPY_CALIB_BYTES (read and write) that calibrates FETCH_SIZE and
    WRITE_SIZE against a known byte count."""
    out = ctx.solve(n_ap)
    log(f"[bench] pmc plan: rounds {out['rounds']} steps {out['total_steps']}")
    n = COPY_CALIB_BYTES // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    log(f"[bench] pmc calibration: 3 copies of {COPY_CALIB_BYTES} bytes (torch.mul by 1.0)")
    print(json.dumps({"pmc_workload": True, "source_sha256": kernel_source_hash(),
                      "copy_bytes": COPY_CALIB_BYTES}), flush=True)


def serving_stream(n_req, rate, seed, log_fn):
    """Seeded request stream shaped like the serving configuration: each
    request is a re-planning solve on a phantom drawn from the tiny /
    prostate / head-and-neck configurations (uniform), with a rigid shift of
    0-5 mm, PTV scale 0.8-1.2 and a budget of 20-50 apertures; arrivals are
    Poisson at `rate` per second.  Phantoms come from a pool of a few seeded
    variants per configuration (generation takes seconds each), every
    request still gets its own context and device copy of D."""
    import numpy as np

    from phantom import make_phantom
    rng = np.random.default_rng(seed)
    pool = {}
    for cfg, nvar in (("tiny", 3), ("prostate", 3), ("headneck", 2)):
        for v in range(nvar):
            shift = rng.uniform(-1.0, 1.0, 3)
            shift = shift / max(1e-9, np.linalg.norm(shift)) * rng.uniform(0.0, 5.0)
            pool[(cfg, v)] = make_phantom(cfg, 100 + v, shift_mm=tuple(shift), ptv_scale=rng.uniform(0.8, 1.2),
                                          dtype="f32")
            log_fn(f"[serve] phantom {cfg}/{v}: {pool[(cfg, v)].n_blt} beamlets, nnz {pool[(cfg, v)].nnz}")
    t = np.cumsum(rng.exponential(1.0 / rate, n_req))
    reqs = []
    for i in range(n_req):
        cfg = ("tiny", "prostate", "headneck")[rng.integers(3)]
        nvar = 2 if cfg == "headneck" else 3
        reqs.append(dict(arrival=float(t[i]), ph=pool[(cfg, int(rng.integers(nvar)))], cfg=cfg,
                         budget=int(rng.integers(20, 51))))
    return reqs


def run_serving(reqs, stream, max_live, cap, sequential, batch_masters=True, **opts):
    """Replay the stream in real time.  Batched: the library's serving loop;
    sequential: one dao_solve at a time in arrival order.  Latency = finish -
    arrival."""
    import numpy as np
    import torch

    import paper_1003_5402_amd as dao
    lat = [None] * len(reqs)
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0   # noqa: E731
    if sequential:
        for i, r in enumerate(reqs):
            while now() < r["arrival"]:
                time.sleep(min(0.005, r["arrival"] - now()))
            ctx = dao.DaoContext.from_phantom(r["ph"], dtype="f32", stream=stream, **opts)
            ctx.solve(r["budget"])
            torch.cuda.synchronize()
            ctx.close()
            lat[i] = now() - r["arrival"]
    else:
        server = dao.Server(max_live=max_live, hbm_cap_bytes=cap, stream=stream, batch_masters=batch_masters)
        nxt, open_t = 0, {}
        while nxt < len(reqs) or open_t:
            while nxt < len(reqs) and reqs[nxt]["arrival"] <= now():
                open_t[server.submit(reqs[nxt]["ph"], reqs[nxt]["budget"], dtype="f32", **opts)] = nxt
                nxt += 1
            if not open_t:
                time.sleep(min(0.005, max(0.0, reqs[nxt]["arrival"] - now())))
                continue
            live, _ = server.step()
            if live == 0:
                time.sleep(0.0005)   # the admission thread is building contexts
            for t in list(open_t):
                state, plan = server.poll(t)
                if state == 2:
                    i = open_t.pop(t)
                    if plan["status"] < 0:
                        raise RuntimeError(f"request {i} failed with status {plan['status']}")
                    lat[i] = now() - reqs[i]["arrival"]
        server.close()
    wall = now()
    lat = np.array(lat)
    return dict(plans_s=len(reqs) / wall, wall_s=wall, p50_s=float(np.percentile(lat, 50)),
                p99_s=float(np.percentile(lat, 99)), mean_s=float(lat.mean()))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="prostate")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--product-iters", type=int, default=200)
    ap.add_argument("--large-config", default="headneck",
                    help="phantom whose products are also timed (D of ~120 MB); 'none' skips it")
    ap.add_argument("--serve-requests", type=int, default=32,
                    help="requests of the serving replay (the serving configuration uses 256)")
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-max-live", type=int, default=8)
    ap.add_argument("--pmc-workload", action="store_true",
                    help="one plan plus a calibration copy, for rocprofv3 --pmc runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the plan is a single-GPU workload "
              "(see DESIGN.md for how it would shard)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1003_5402_amd as dao
    from phantom import make_phantom

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a HIP device")
    log(f"[bench] phantom {args.config} seed {args.seed}")
    ph = make_phantom(args.config, args.seed)
    stream = torch.cuda.current_stream().cuda_stream
    t0 = time.perf_counter()
    ctx = dao.DaoContext.from_phantom(ph, stream=stream)
    create_s = time.perf_counter() - t0
    info = ctx.info()
    n_ap = ph.n_apertures
    log(f"[bench] ctx ready in {create_s:.2f} s: {info}")
    if args.pmc_workload:
        pmc_workload(ctx, n_ap, torch)
        ctx.close()
        return

    for w in range(args.warmup):
        out = ctx.solve(n_ap)
        log(f"[bench] warmup {w}: rounds {out['rounds']} steps {out['total_steps']} F {out['F']:.6e}")
    torch.cuda.synchronize()
    lat = []
    outs = []
    t_start = time.perf_counter()
    for k in range(args.steps):
        t0 = time.perf_counter()
        out = ctx.solve(n_ap)
        lat.append(time.perf_counter() - t0)
        outs.append(out)
        log(f"[bench] plan {k}: {lat[-1]:.4f} s rounds {out['rounds']} steps {out['total_steps']} "
            f"ls {out['total_ls_evals']} F {out['F']:.8e}")
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    lat = np.array(lat)

    # master kernels: one instrumented plan per kernel, every launch bracketed
    # by HIP events on the context stream; algorithmic bytes counted on the
    # device.  Plans are deterministic, so each instrumented plan repeats
    # exactly the launches of a timed plan.
    kernels = {}
    try:
        ctx.profile_start(4)
        ctx.profile_stop()
        plist = [(4, "k_master_coop")]
    except dao.DaoError:
        plist = [(0, "k_upd_ap"), (1, "k_qstep_ap"), (2, "k_lseval_ap"), (3, "k_dir_ap")]
    for kid, kname in plist:
        ctx.profile_start(kid)
        ctx.solve(n_ap)
        r = ctx.profile_stop()
        r["avg_us"] = r["total_us"] / max(1, r["launches"])
        r["GBs"] = r["total_bytes"] / max(r["total_us"], 1e-9) / 1e3
        if kid == 4:
            r["phases_us"] = ctx.profile_phases()
            log(f"[bench] {kname} phases (us per plan): {r['phases_us']}")
        kernels[kname] = r
        log(f"[bench] {kname}: {r['launches']} launches ({r['working_launches']} working), "
            f"{r['total_us'] / 1e3:.1f} ms, avg {r['avg_us']:.2f} us, {r['GBs']:.0f} GB/s")
    dom = max(kernels, key=lambda k: kernels[k]["total_us"])
    dk_ = kernels[dom]
    traffic = measured_traffic(dom, args.config)

    # the plain products (the kernels behind dao_dose / dao_gradient)
    us_dose = ctx.time_product(0, args.product_iters)
    us_grad = ctx.time_product(1, args.product_iters)
    gbs_dose = info["bytes_dose"] / (us_dose * 1e-6) / 1e9
    gbs_grad = info["bytes_gradient"] / (us_grad * 1e-6) / 1e9
    log(f"[bench] D x: {us_dose:.2f} us {gbs_dose:.0f} GB/s; D^T u: {us_grad:.2f} us {gbs_grad:.0f} GB/s")
    # cold: a 1 GiB read (4x the last-level cache) before every timed launch
    scrub = torch.zeros(1 << 30, dtype=torch.uint8, device="cuda")
    cold_iters = max(1, args.product_iters // 10)
    us_dose_c = ctx.time_product_cold(0, cold_iters, scrub)
    us_grad_c = ctx.time_product_cold(1, cold_iters, scrub)
    # every product variant, forced (the tuned choice above is one of them)
    variants = {}
    for dv, gd in ((0, 4), (1, 8), (2, 16), (3, 4)):
        vc = dao.DaoContext.from_phantom(ph, dtype="f32", stream=stream, product_tune=0, dose_variant=dv,
                                         gradient_depth=gd)
        variants[f"dose{dv}_depth{gd}"] = {
            "dose_us": vc.time_product(0, args.product_iters), "gradient_us": vc.time_product(1, args.product_iters),
            "dose_cold_us": vc.time_product_cold(0, cold_iters, scrub),
            "gradient_cold_us": vc.time_product_cold(1, cold_iters, scrub)}
        vc.close()
    log(f"[bench] product variants (tuned: dose {info['dose_variant']}, depth {info['gradient_depth']}): {variants}")
    # the same products on the larger phantom (D several times the size, nearer
    # the streaming regime the kernels are built for)
    large = None
    if args.large_config != "none" and args.large_config != args.config:
        phl = make_phantom(args.large_config, args.seed)
        large = {"phantom": args.large_config, "nnz": int(phl.row_ptr[-1]), "n_blt": int(phl.n_blt)}
        for fname, fmt in (("f32", dao.DAO_DFMT_NATIVE), ("f16", dao.DAO_DFMT_F16)):
            lc = dao.DaoContext.from_phantom(phl, dtype="f32", stream=stream, d_format=fmt)
            li = lc.info()
            ud, ug = lc.time_product(0, args.product_iters), lc.time_product(1, args.product_iters)
            udc, ugc = lc.time_product_cold(0, cold_iters, scrub), lc.time_product_cold(1, cold_iters, scrub)
            large[fname] = {
                "dose_bytes": li["bytes_dose"], "gradient_bytes": li["bytes_gradient"],
                "dose_us": ud, "gradient_us": ug, "dose_cold_us": udc, "gradient_cold_us": ugc,
                "dose_GBs": li["bytes_dose"] / (ud * 1e-6) / 1e9, "gradient_GBs": li["bytes_gradient"] / (ug * 1e-6) / 1e9,
                "dose_cold_GBs": li["bytes_dose"] / (udc * 1e-6) / 1e9,
                "gradient_cold_GBs": li["bytes_gradient"] / (ugc * 1e-6) / 1e9,
                "dose_frac_cold": li["bytes_dose"] / (udc * 1e-6) / 1e9 / HBM_PEAK_GBS,
                "gradient_frac_cold": li["bytes_gradient"] / (ugc * 1e-6) / 1e9 / HBM_PEAK_GBS,
                "tuned": {"dose_variant": li["dose_variant"], "gradient_depth": li["gradient_depth"]}}
            lc.close()
            log(f"[bench] {args.large_config} {fname} products: {large[fname]}")
        del phl
    del scrub
    gbs_dose_c = info["bytes_dose"] / (us_dose_c * 1e-6) / 1e9
    gbs_grad_c = info["bytes_gradient"] / (us_grad_c * 1e-6) / 1e9
    log(f"[bench] cold D x: {us_dose_c:.2f} us {gbs_dose_c:.0f} GB/s; "
        f"cold D^T u: {us_grad_c:.2f} us {gbs_grad_c:.0f} GB/s")

    # 16-bit storage of D (FP16 / BF16 value per beamlet scale, optional FP16
    # residual): product throughput and one plan each, on the same phantom
    reduced = {}
    scrub = torch.zeros(1 << 30, dtype=torch.uint8, device="cuda")
    for fname, fmt in (("f16", dao.DAO_DFMT_F16), ("bf16", dao.DAO_DFMT_BF16)):
        for res in (0, 1):
            rc = dao.DaoContext.from_phantom(ph, dtype="f32", stream=stream, d_format=fmt, d_residual=res)
            ri = rc.info()
            ud, ug = rc.time_product(0, args.product_iters), rc.time_product(1, args.product_iters)
            udc, ugc = rc.time_product_cold(0, cold_iters, scrub), rc.time_product_cold(1, cold_iters, scrub)
            rc.solve(n_ap)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ro = rc.solve(n_ap)
            torch.cuda.synchronize()
            pt = time.perf_counter() - t0
            key = f"{fname}{'+lo' if res else ''}"
            reduced[key] = {
                "dose_us": ud, "dose_bytes": ri["bytes_dose"], "dose_GBs": ri["bytes_dose"] / (ud * 1e-6) / 1e9,
                "gradient_us": ug, "gradient_bytes": ri["bytes_gradient"],
                "gradient_GBs": ri["bytes_gradient"] / (ug * 1e-6) / 1e9,
                "dose_cold_us": udc, "gradient_cold_us": ugc,
                "dose_speedup_vs_f32": us_dose / ud, "gradient_speedup_vs_f32": us_grad / ug,
                "plan_s": pt, "plan_F": ro["F"], "plan_F_rel_vs_f32": (ro["F"] - outs[-1]["F"]) / outs[-1]["F"],
                "device_bytes": ri["device_bytes"],
            }
            log(f"[bench] D {key}: D x {ud:.2f} us ({reduced[key]['dose_GBs']:.0f} GB/s), D^T u {ug:.2f} us "
                f"({reduced[key]['gradient_GBs']:.0f} GB/s), plan {pt:.4f} s F {ro['F']:.8e}")
            rc.close()
    del scrub

    # serving: the same seeded request stream replayed batched (FP32 D and
    # FP16 D) and as sequential plain solves
    serve = None
    if args.serve_requests > 0:
        reqs = serving_stream(args.serve_requests, args.serve_rate, args.seed, log)
        cap = 64 << 30
        serve = dict(requests=args.serve_requests, rate_per_s=args.serve_rate, max_live=args.serve_max_live,
                     hbm_cap_bytes=cap,
                     mix={c: sum(r["cfg"] == c for r in reqs) for c in ("tiny", "prostate", "headneck")})
        serve["batched_f32"] = run_serving(reqs, stream, args.serve_max_live, cap, False)
        log(f"[bench] serving batched FP32: {serve['batched_f32']}")
        serve["interleaved_f32"] = run_serving(reqs, stream, args.serve_max_live, cap, False, batch_masters=False)
        log(f"[bench] serving interleaved FP32 (masters one after another): {serve['interleaved_f32']}")
        serve["batched_f16"] = run_serving(reqs, stream, args.serve_max_live, cap, False,
                                           d_format=dao.DAO_DFMT_F16)
        log(f"[bench] serving batched FP16 D: {serve['batched_f16']}")
        serve["sequential_f32"] = run_serving(reqs, stream, 1, cap, True)
        log(f"[bench] serving sequential FP32: {serve['sequential_f32']}")
        serve["speedup_plans_s"] = serve["batched_f32"]["plans_s"] / serve["sequential_f32"]["plans_s"]
        serve["speedup_interleaved_plans_s"] = (serve["interleaved_f32"]["plans_s"] /
                                                serve["sequential_f32"]["plans_s"])

    steps_per_plan = int(outs[-1]["total_steps"])
    result = {
        "metric": METRIC,
        "value": args.steps / total,
        "unit": "plans/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"prostate-shaped phantom {ph.shape[0]}x{ph.shape[1]}x{ph.shape[2]} voxels at 2.5 mm, "
                         f"{ph.n_beams} beams, {ph.n_blt} beamlets, nnz {ph.nnz}, {n_ap}-aperture plan, "
                         f"FP32 dose matrix"),
            "phantom": args.config, "seed": args.seed, "apertures": n_ap,
            "n_vox_nonempty": info["n_vox_nonempty"], "nnz": info["nnz"], "n_blt": info["n_blt"],
        },
        "plan_s_p50": float(np.percentile(lat, 50)),
        "plan_s_p99": float(np.percentile(lat, 99)),
        "plan_s_mean": float(lat.mean()),
        "plan_split_s": {"pricing": float(np.mean([o["price_s"] for o in outs])),
                         "columns_and_master": float(np.mean([o["master_s"] for o in outs]))},
        "master_steps_per_plan": steps_per_plan,
        "ls_evals_per_plan": int(outs[-1]["total_ls_evals"]),
        "final_F": outs[-1]["F"],
        "create_s": create_s,
        "products": {
            "dose_us": us_dose, "dose_bytes": info["bytes_dose"], "dose_GBs": gbs_dose,
            "gradient_us": us_grad, "gradient_bytes": info["bytes_gradient"], "gradient_GBs": gbs_grad,
            "dose_cold_us": us_dose_c, "dose_cold_GBs": gbs_dose_c,
            "gradient_cold_us": us_grad_c, "gradient_cold_GBs": gbs_grad_c,
            "dose_frac_cold": gbs_dose_c / HBM_PEAK_GBS, "gradient_frac_cold": gbs_grad_c / HBM_PEAK_GBS,
            "tuned": {"dose_variant": info["dose_variant"], "gradient_depth": info["gradient_depth"]},
            "variants": variants,
            "note": ("D x = k_dose, D^T u = k_gradT, timed standalone: warm back-to-back (D fits the 256 MB "
                     "last-level cache) and cold (1 GiB scrub read before each timed launch)"),
        },
        "products_large": large,
        "master_kernels": kernels,
        "d_16bit": reduced,
        "serving": serve,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": dk_["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": dk_["GBs"] / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_launch": dk_["total_bytes"] / max(1, dk_["launches"]),
                     "us_per_launch": dk_["avg_us"], "launches_per_plan": dk_["launches"]},
    }
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(ph, steps_per_plan, int(outs[-1]["rounds"]), args.cpu_seconds)
    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
