"""Benchmark: time-to-50-aperture plan on one GPU.

One "step" is one whole plan: dao_solve from an empty pool to 50 apertures
(pricing, master, column generation) with the dose matrix resident on the
device.  The headline workload is the head-and-neck-shaped phantom (the
largest configuration); the prostate-shaped plan is timed beside it.  Prints
one JSON line.

    python bench.py [--steps K] [--warmup W] [--config headneck] [--cpu-seconds S]
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
    master step and per pricing round are extrapolated to one whole plan with
    the master step count the plan takes (the GPU runs the same algorithm).
    """
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    from oracle.master import MasterState, solve_master

    with threadpool_limits(limits=1):
        D = ph.csr()
        if ph.dtype == "f32":   # the problem the FP32 context holds
            D = D.copy()
            D.data = D.data.astype(np.float32).astype(np.float64)
        P = oracle.make_problem(D, ph.rows_per_beam, ph.row_len, ph.vox_struct, ph.prescriptions)
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
                sample=(f"FP64 oracle column generation on the same phantom for its first {rounds} rounds "
                        f"({steps} master steps, {t_master + t_price:.1f} s); {s_step * 1e3:.1f} ms per "
                        f"master step and {s_round * 1e3:.1f} ms per pricing round extrapolated to the "
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


def pmc_workload(ctx, n_ap, torch, what="plan"):
    """Short run for counter collection: one plan (or, with what="products",
    8 cold launches of each sparse product after a cache scrub), then a plain
    device copy of COPY_CALIB_BYTES (read and write) that calibrates
    FETCH_SIZE and WRITE_SIZE against a known byte count."""
    if what == "products":
        scrub = torch.zeros(1 << 30, dtype=torch.uint8, device="cuda")
        for kernel in (0, 1):
            us = ctx.time_product_cold(kernel, 8, scrub)
            log(f"[bench] pmc product {kernel}: 8 cold launches, {us:.2f} us each")
        del scrub
    else:
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


def release_device(torch):
    """Hand torch's cached device memory back before the interpreter exits,
    so that no device allocation is left for the runtime's teardown (the
    library's contexts are closed by then)."""
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


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


def time_plans(dao, ph, stream, steps, warmup, **opts):
    """K timed plans (after W warm-ups) on one context; returns the context
    and the figures."""
    import numpy as np
    import torch
    ctx = dao.DaoContext.from_phantom(ph, stream=stream, **opts)
    n_ap = ph.n_apertures
    for w in range(warmup):
        out = ctx.solve(n_ap)
        log(f"[bench] {ph.name} warmup {w}: rounds {out['rounds']} steps {out['total_steps']} F {out['F']:.6e}")
    torch.cuda.synchronize()
    lat, outs = [], []
    t_start = time.perf_counter()
    for k in range(steps):
        t0 = time.perf_counter()
        out = ctx.solve(n_ap)
        lat.append(time.perf_counter() - t0)
        outs.append(out)
        log(f"[bench] {ph.name} plan {k}: {lat[-1]:.4f} s rounds {out['rounds']} steps {out['total_steps']} "
            f"ls {out['total_ls_evals']} F {out['F']:.8e}")
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    lat = np.array(lat)
    o = outs[-1]
    fig = {
        "plans_s": steps / total, "total_s": total,
        "plan_s_p50": float(np.percentile(lat, 50)), "plan_s_p99": float(np.percentile(lat, 99)),
        "plan_s_mean": float(lat.mean()),
        "plan_split_s": {"pricing": float(np.mean([x["price_s"] for x in outs])),
                         "columns_and_master": float(np.mean([x["master_s"] for x in outs]))},
        "rounds": int(o["rounds"]), "master_steps_per_plan": int(o["total_steps"]),
        "ls_evals_per_plan": int(o["total_ls_evals"]),
        "round_steps": [int(v) for v in o["round_steps"]], "capped_rounds": int(o["capped_rounds"]),
        "final_F": o["F"], "master_form": ctx.info()["last_master_form"],
    }
    return ctx, fig


def profile_master(dao, ctx, n_ap, algo_step_bytes, ls_pass_bytes):
    """One instrumented plan: every launch of the master kernel bracketed by
    HIP events on the context stream.  Plans are deterministic, so it repeats
    the launches of a timed plan.  Algorithmic bytes per launch follow the
    per-step count: two beamlet products plus the line-search passes."""
    try:
        ctx.profile_start(4)
        ctx.profile_stop()
        plist = [(4, "k_master_coop")]
    except dao.DaoError:
        plist = [(0, "k_upd_ap"), (1, "k_qstep_ap"), (2, "k_lseval_ap"), (3, "k_dir_ap")]
    kernels = {}
    for kid, kname in plist:
        ctx.profile_start(kid)
        out = ctx.solve(n_ap)
        r = ctx.profile_stop()
        r["avg_us"] = r["total_us"] / max(1, r["launches"])
        r["steps_per_plan"] = int(out["total_steps"])
        r["ls_evals_per_plan"] = int(out["total_ls_evals"])
        r["algo_bytes_per_plan"] = out["total_steps"] * algo_step_bytes + out["total_ls_evals"] * ls_pass_bytes
        r["algo_GBs"] = r["algo_bytes_per_plan"] / max(r["total_us"], 1e-9) / 1e3
        if kid == 4:
            r["phases_us"] = ctx.profile_phases()
            log(f"[bench] {kname} phases (us per plan): {r['phases_us']}")
        kernels[kname] = r
        log(f"[bench] {kname}: {r['launches']} launches ({r['working_launches']} working), "
            f"{r['total_us'] / 1e3:.2f} ms, avg {r['avg_us']:.2f} us, {r['algo_GBs']:.0f} GB/s algorithmic")
    return kernels


def read_at_size(ctx, torch, nbytes, scrub, iters=10):
    """A plain streaming read of `nbytes` (the library's 16-byte grid-stride
    read kernel, dao_time_read_cold), cold exactly as the products are timed:
    the practical ceiling for a kernel that reads that many bytes once,
    launch ramp and drain included.  Returns GB/s."""
    n = (int(nbytes) + 15) // 16 * 16
    x = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    us = ctx.time_read_cold(x, n, iters, scrub)
    del x
    return n / (us * 1e-6) / 1e9


def time_products(ctx, info, iters, scrub, torch=None):
    """k_dose / k_gradT (the kernels behind dao_dose / dao_gradient): warm
    back to back, and cold after a 1 GiB scrub read before every launch;
    with `torch`, also the cold streaming-read rate at each product's byte
    count."""
    cold_iters = max(1, iters // 10)
    ud, ug = ctx.time_product(0, iters), ctx.time_product(1, iters)
    udc, ugc = ctx.time_product_cold(0, cold_iters, scrub), ctx.time_product_cold(1, cold_iters, scrub)
    bd, bg = info["bytes_dose"], info["bytes_gradient"]
    extra = {}
    if torch is not None:
        rd, rg = read_at_size(ctx, torch, bd, scrub), read_at_size(ctx, torch, bg, scrub)
        extra = {"read_cold_GBs_at_dose_bytes": rd, "read_cold_GBs_at_gradient_bytes": rg,
                 "dose_cold_vs_read": bd / (udc * 1e-6) / 1e9 / rd,
                 "gradient_cold_vs_read": bg / (ugc * 1e-6) / 1e9 / rg}
    return {**extra, "dose_bytes": bd, "gradient_bytes": bg, "dose_us": ud, "gradient_us": ug,
            "dose_cold_us": udc, "gradient_cold_us": ugc,
            "dose_GBs": bd / (ud * 1e-6) / 1e9, "gradient_GBs": bg / (ug * 1e-6) / 1e9,
            "dose_cold_GBs": bd / (udc * 1e-6) / 1e9, "gradient_cold_GBs": bg / (ugc * 1e-6) / 1e9,
            "dose_frac_cold": bd / (udc * 1e-6) / 1e9 / HBM_PEAK_GBS,
            "gradient_frac_cold": bg / (ugc * 1e-6) / 1e9 / HBM_PEAK_GBS,
            "tuned": {"dose_variant": info["dose_variant"], "gradient_depth": info["gradient_depth"]}}


def copy_ceiling(torch):
    """Achievable HBM bandwidth: a 1 GiB device copy (read + write bytes over
    the time of the copy), best of 5."""
    n = 1 << 28
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    best = 0.0
    for _ in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        best = max(best, 2.0 * n * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del src, dst
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="headneck")
    ap.add_argument("--also", default="prostate", help="second phantom whose plan is timed beside; 'none' skips")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--product-iters", type=int, default=200)
    ap.add_argument("--serve-requests", type=int, default=256,
                    help="requests of the serving replay (the serving configuration uses 256)")
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-max-live", type=int, default=8)
    ap.add_argument("--pmc-workload", nargs="?", const="plan", default=None, choices=["plan", "products"],
                    help="one plan (or cold product launches) plus a calibration copy, for rocprofv3 --pmc runs")
    ap.add_argument("--round-log", default=None,
                    help="append the per-round records of one untimed headline plan to this JSON-lines file")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: one plan's dose matrix, aperture dose matrix and master "
              "state fit one GPU, and several GPUs are not measured", file=sys.stderr)
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
    n_ap = ph.n_apertures
    if args.pmc_workload:
        ctx = dao.DaoContext.from_phantom(ph, stream=stream)
        pmc_workload(ctx, n_ap, torch, args.pmc_workload)
        ctx.close()
        release_device(torch)
        return

    t0 = time.perf_counter()
    ctx, plan = time_plans(dao, ph, stream, args.steps, args.warmup)
    info = ctx.info()
    create_s = time.perf_counter() - t0
    log(f"[bench] {args.config}: {plan['plans_s']:.3f} plans/s, {plan['master_steps_per_plan']} steps, "
        f"capped rounds {plan['capped_rounds']}, form {plan['master_form']}")
    if args.round_log:
        ctx.solve(n_ap, round_log=args.round_log)   # untimed: the timed plans are deterministic

    # the master kernel, with the algorithmic bytes of a master step: one
    # forward and one transposed beamlet product, and per line-search
    # evaluation one pass over d (8 B), q (4 B) and the structure class (1 B)
    step_bytes = info["bytes_dose"] + info["bytes_gradient"]
    ls_bytes = info["n_vox_nonempty"] * (8 + 4 + 1)
    kernels = profile_master(dao, ctx, n_ap, step_bytes, ls_bytes)
    dom = max(kernels, key=lambda k: kernels[k]["total_us"])
    dk_ = kernels[dom]
    traffic = measured_traffic(dom, args.config)
    hbm_copy = copy_ceiling(torch)
    log(f"[bench] device copy: {hbm_copy:.0f} GB/s")

    scrub = torch.zeros(1 << 30, dtype=torch.uint8, device="cuda")
    products = time_products(ctx, info, args.product_iters, scrub, torch)
    log(f"[bench] {args.config} products: {products}")

    # the precision form: D stored in 16 bits (FP16 / BF16 values over a
    # per-beamlet FP32 scale, optional FP16 residual) and the aperture dose
    # matrix in FP16 (or FP32): products and timed plans, same phantom
    reduced = {}
    combos = [("f16", dao.DAO_DFMT_F16, 0, 1), ("f16", dao.DAO_DFMT_F16, 1, 1), ("bf16", dao.DAO_DFMT_BF16, 0, 1),
              ("bf16", dao.DAO_DFMT_BF16, 1, 1), ("f16", dao.DAO_DFMT_F16, 0, 0), ("f32", dao.DAO_DFMT_NATIVE, 0, 1)]
    for fname, fmt, res, dk16 in combos:
        if True:
            rc = dao.DaoContext.from_phantom(ph, dtype="f32", stream=stream, d_format=fmt, d_residual=res,
                                             dk_format=dao.DAO_DFMT_F16 if dk16 else dao.DAO_DFMT_NATIVE)
            ri = rc.info()
            key = f"{fname}{'+lo' if res else ''}{'_dk16' if dk16 else '_dk32'}"
            reduced[key] = time_products(rc, ri, args.product_iters, scrub)
            rc.solve(n_ap)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            nrep = 5
            for _ in range(nrep):
                ro = rc.solve(n_ap)
            torch.cuda.synchronize()
            pt = (time.perf_counter() - t0) / nrep
            reduced[key].update(plan_s=pt, plan_F=ro["F"], plan_F_rel_vs_f32=(ro["F"] - plan["final_F"]) / plan["final_F"],
                                plan_steps=int(ro["total_steps"]), device_bytes=ri["device_bytes"])
            log(f"[bench] D {key}: {reduced[key]}")
            rc.close()

    # the second phantom's plan and products
    also = None
    if args.also != "none" and args.also != args.config:
        pha = make_phantom(args.also, args.seed)
        actx, also = time_plans(dao, pha, stream, args.steps, args.warmup)
        ainfo = actx.info()
        also["config"] = {"phantom": args.also, "n_vox_nonempty": ainfo["n_vox_nonempty"], "nnz": ainfo["nnz"],
                          "n_blt": ainfo["n_blt"], "apertures": pha.n_apertures}
        akern = profile_master(dao, actx, pha.n_apertures, ainfo["bytes_dose"] + ainfo["bytes_gradient"],
                               ainfo["n_vox_nonempty"] * 13)
        also["master_kernels"] = akern
        also["products"] = time_products(actx, ainfo, args.product_iters, scrub, torch)
        actx.close()
        log(f"[bench] {args.also}: {also['plans_s']:.3f} plans/s")
        del pha
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
        # the precision form: FP16 D with the selective residual (final rounds
        # and near-tie pricing with the FP16 residual) and D_K in FP16 where
        # the master streams it (automatic storage)
        f16_opts = dict(d_format=dao.DAO_DFMT_F16, d_residual=2, dk_format=dao.DAO_DFMT_AUTO)
        serve["f16_options"] = {"d_format": "f16", "d_residual": "selective", "dk_format": "auto"}
        serve["batched_f16"] = run_serving(reqs, stream, args.serve_max_live, cap, False, **f16_opts)
        log(f"[bench] serving batched FP16 D + automatic D_K (selective residual): {serve['batched_f16']}")
        serve["sequential_f32"] = run_serving(reqs, stream, 1, cap, True)
        log(f"[bench] serving sequential FP32: {serve['sequential_f32']}")
        # capacity: the same requests all queued at once, so that plans/s is
        # set by the server rather than by the arrival rate
        sat = [dict(r, arrival=0.0) for r in reqs]
        serve["saturated_f32"] = run_serving(sat, stream, args.serve_max_live, cap, False)
        log(f"[bench] serving saturated FP32: {serve['saturated_f32']}")
        serve["saturated_f16"] = run_serving(sat, stream, args.serve_max_live, cap, False, **f16_opts)
        log(f"[bench] serving saturated FP16 D + automatic D_K (selective residual): {serve['saturated_f16']}")
        serve["saturated_dk_auto"] = run_serving(sat, stream, args.serve_max_live, cap, False,
                                                 dk_format=dao.DAO_DFMT_AUTO)
        log(f"[bench] serving saturated FP32 D + automatic D_K: {serve['saturated_dk_auto']}")
        serve["speedup_plans_s"] = serve["batched_f32"]["plans_s"] / serve["sequential_f32"]["plans_s"]
        serve["speedup_f16_plans_s"] = serve["batched_f16"]["plans_s"] / serve["sequential_f32"]["plans_s"]
        serve["saturated_f16_vs_f32"] = serve["saturated_f16"]["plans_s"] / serve["saturated_f32"]["plans_s"]
        serve["saturated_dk_auto_vs_f32"] = serve["saturated_dk_auto"]["plans_s"] / serve["saturated_f32"]["plans_s"]

    algo_per_launch = dk_["algo_bytes_per_plan"] / max(1, dk_["launches"])
    result = {
        "metric": METRIC,
        "value": plan["plans_s"],
        "unit": "plans/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * plan["total_s"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{args.config} phantom {ph.shape[0]}x{ph.shape[1]}x{ph.shape[2]} voxels at 2.5 mm, "
                         f"{ph.n_beams} beams, {ph.n_blt} beamlets, nnz {ph.nnz}, {n_ap}-aperture plan, "
                         f"FP32 dose matrix"),
            "phantom": args.config, "seed": args.seed, "apertures": n_ap,
            "n_vox_nonempty": info["n_vox_nonempty"], "nnz": info["nnz"], "n_blt": info["n_blt"],
        },
        "create_s": create_s,
        "plan": {k: v for k, v in plan.items() if k not in ("plans_s", "total_s")},
        "products": products,
        "hbm_copy_GBs": hbm_copy,
        "master_kernels": kernels,
        "d_16bit": reduced,
        args.also: also,
        "serving": serve,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": algo_per_launch / (dk_["avg_us"] * 1e-6) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": algo_per_launch / (dk_["avg_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS,
                     "traffic": traffic, "algo_bytes_per_launch": algo_per_launch,
                     "us_per_launch": dk_["avg_us"], "launches_per_plan": dk_["launches"],
                     "copy_GBs": hbm_copy,
                     "note": ("algorithmic bytes of a master step: one forward and one transposed beamlet "
                              "product plus 13 B per non-empty voxel row per line-search evaluation")},
    }
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(ph, plan["master_steps_per_plan"], plan["rounds"], args.cpu_seconds)
    ctx.close()
    release_device(torch)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
