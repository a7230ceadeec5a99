"""Benchmark: all-to-all CCM pairs/s on one MI355X.

Default workload (one step = the whole hot path once): 10000 calcium-like
series of L = 2000 samples (AR(1)-filtered Poisson spike trains, 2000 of them
modulated by 20 latent logistic drivers), float32; the simplex E sweep
E = 1..20 (Tp = 1) selects every series' E*, then the full 10000 x 10000
cross map (Tp = 0) builds each library's table once per E* in use and looks
up every target.  value = 10^8 pairs / step time of the chosen form; the
plain form is timed on the same steps for the ratio.

Prints one JSON line.  Besides the driver's fields it carries:
* kernels: per kernel family of the timed chosen-form steps, the HIP-event
  time per step (events recorded around every launch on the library's stream)
  and the family's algorithmic work per step with its fraction of the unit
  that bounds it;
* roofline: the same for the dominant family (the one with the most time);
  traffic comes from rocprofv3 counters recorded for the current kernel
  source (null when the source changed since);
* cpu_baseline: the CPU oracle timed on the host cores on 16/10000 of the
  step (16 series' E sweeps and 16 libraries' full cross-map rows);
* parity: rho of those rows and sweeps against the oracle, E* with the
  near-tie rule, and the libraries' kNN tables bit for bit.

Other workloads (--workload): network (1024 x 5000 logistic network), uneven
(batched plan on 4096 series of uneven length), learned (network-selected E on
100000 series), twokernel (materialised distance matrix vs fused kNN).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks.  The vector ALU figure is one fp32 op per lane per
# clock (256 CUs x 128 lanes x 2.4 GHz); the 157.3 TFLOP/s headline counts a
# fused multiply-add as two flops and none of the neighbour key's operations
# fuse.
PEAK = {
    "hbm": (8.0e12, "GB/s", 1e9),
    "mfma": (2.5e15, "TFLOP/s", 1e12),   # dense BF16 matrix cores
    "alu": (256 * 128 * 2.4e9, "Top/s", 1e12),
}

CALCIUM = dict(N=10000, L=2000, E_max=20, tau=1, seed=4)
NETWORK = dict(N=1024, L=5000, E_max=20, tau=1, seed=2)

# E groups of the batched scans (the kernels' own grouping).
EXACT_GROUPS = ((1, 8), (9, 12), (13, 15), (16, 18), (19, 20))
CHOSEN_EXACT = ((1, 4),)
FILTER_GROUPS = ((5, 8), (9, 11), (12, 13), (14, 16), (17, 18), (19, 20))

FAMILY_SOURCE = {
    "lookup": "paper_2105_12301_amd/csrc/lookup.hip",
    "filter_scan": "paper_2105_12301_amd/csrc/gram.hip",
    "batched_scan": "paper_2105_12301_amd/csrc/sweep_multi.hip",
    "exact_scan": "paper_2105_12301_amd/csrc/knn.hip",
    "distances": "paper_2105_12301_amd/csrc/twokernel.hip",
    "row_topk": "paper_2105_12301_amd/csrc/twokernel.hip",
}


# ------------------------------------------------------ algorithmic work --
def _m(L, E, Tp):
    return L - (E - 1) - Tp


def scan_ops_exact(N, L, Es, Tp):
    """VALU ops of one exact scan per (series, E): every ordered pair q != p
    of the m query points costs E subtractions, E multiplies, E adds and one
    compare (the float32 key of Algorithm 1 and its top-k test)."""
    tot = 0
    for E in Es:
        m = _m(L, E, Tp)
        if m - 1 >= E + 1:
            tot += N * m * (m - 1) * (3 * E + 1)
    return tot


def scan_ops_grouped(N, L, groups, Tp, E_max=20):
    """VALU ops of the batched exact scan: one running key per pair and group
    costs 3 ops per lag up to the group's largest E plus one compare per E of
    the group (pairs counted at the group's smallest E)."""
    tot = 0
    for lo, hi in groups:
        hi = min(hi, E_max)
        if lo > hi:
            continue
        m = _m(L, lo, Tp)
        tot += N * m * (m - 1) * (3 * hi + (hi - lo + 1))
    return tot


def gram_flops(N, L, Tp, groups=FILTER_GROUPS, E_max=20):
    """Matrix-core work of the filtered scans: the Gram product of the group's
    largest E, 2 E_hi flops per ordered pair (multiply and add per lag)."""
    tot = 0
    for lo, hi in groups:
        hi = min(hi, E_max)
        if lo > hi:
            continue
        m = _m(L, lo, Tp)
        tot += 2 * hi * N * m * (m - 1)
    return tot


def lookup_bytes(N_lib, L, E_of_targets):
    """Algorithmic bytes of the lookups: every pair reads its target once
    (4 L bytes) and writes rho (4 bytes); every (library, E in use) reads its
    table once (8 m k bytes: int32 index + float32 weight per neighbour)."""
    counts = np.bincount(np.asarray(E_of_targets, dtype=np.int64), minlength=21)
    tot = 0
    for E in range(1, 21):
        c = int(counts[E])
        if c == 0:
            continue
        m = _m(L, E, 0)
        tot += N_lib * c * (4 * L + 4) + N_lib * 8 * m * (E + 1)
    return tot


# ------------------------------------------------------------- traffic --
def recorded_traffic(family):
    """HBM bytes per step of a kernel family from the rocprofv3 counter
    summaries under profiles/ (lines 'bench-traffic: family=F sha256=S
    bytes_per_step=B workload=W'), kept only while the kernel source still
    has that hash."""
    src = FAMILY_SOURCE.get(family)
    pdir = os.path.join(ROOT, "profiles")
    if not src or not os.path.isdir(pdir):
        return None
    with open(os.path.join(ROOT, src), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    pat = re.compile(r"bench-traffic: family=(\S+) sha256=(\S+) bytes_per_step=(\S+) workload=(\S+)")
    for name in sorted(os.listdir(pdir)):
        if not name.endswith((".md", ".txt")):
            continue
        with open(os.path.join(pdir, name)) as f:
            for line in f:
                mt = pat.search(line)
                if mt and mt.group(1) == family and mt.group(2) == sha:
                    return {"bytes_per_step": float(mt.group(3)), "workload": mt.group(4),
                            "source": f"profiles/{name}"}
    return None


# ---------------------------------------------------------------- CPU leg --
_CPU = {}


def _cpu_init(X):
    os.environ["OMP_NUM_THREADS"] = "1"
    _CPU["X"] = X


def _cpu_ready(_):
    time.sleep(0.3)
    return os.getpid()


def _cpu_sweep_task(args):
    s, E_max = args
    from oracle import edm_oracle as O
    X = _CPU["X"]
    L = X.shape[1]
    rho, E_opt = O.simplex_sweep(X[s:s + 1], [L], E_max, tau=1, Tp=1)
    return ("sweep", s, rho[0], int(E_opt[0]))


def _cpu_row_task(args):
    i, E_star = args
    from oracle import edm_oracle as O
    X = _CPU["X"]
    N, L = X.shape
    # the oracle's CCM row (Section 3.4: one table per E in use, every target
    # of that E looked up through it), keeping a digest of each table
    rho = np.full(N, np.nan)
    hashes = {}
    for E in sorted(set(int(e) for e in E_star if e >= 1)):
        idx, _ = O.knn(X[i], E, 1, 0)
        _, wbar = O.weights(X[i], idx, E, 1)
        hashes[E] = hashlib.sha1(np.ascontiguousarray(idx, dtype=np.int32).tobytes()).hexdigest()
        for j in np.nonzero(E_star == E)[0]:
            yhat, obs = O.lookup(idx, wbar, X[j], E, 1, 0)
            rho[j] = O.pearson(obs, yhat)
    return ("row", i, rho, hashes)


def cpu_leg(X, sweep_series, rows, E_star, E_max, cores):
    """The oracle on 16 series' sweeps and 16 libraries' full rows, spread
    over `cores` single-threaded spawned workers; returns (wall seconds of the
    work, results).  Worker start-up and the data hand-over are not timed."""
    import multiprocessing as mp

    ctx = mp.get_context("spawn")
    tasks = [(_cpu_sweep_task, (int(s), E_max)) for s in sweep_series]
    tasks += [(_cpu_row_task, (int(i), E_star)) for i in rows]
    pool = ctx.Pool(cores, initializer=_cpu_init, initargs=(X,))
    try:
        pool.map(_cpu_ready, range(cores), chunksize=1)
        t0 = time.perf_counter()
        pending = [pool.apply_async(fn, (a,)) for fn, a in tasks]
        out = [p.get() for p in pending]
        wall = time.perf_counter() - t0
    finally:
        pool.close()
        pool.join()
    return wall, out


# ---------------------------------------------------------------- GPU leg --
def run_form(torch, edm, ctx, Xd, rho, E_max, steps, warmup, form, timing):
    """Time `steps` steps of one form after `warmup` untimed ones.  The chosen
    form runs the step as one edm_sweep_ccm call (its cross-map tables come
    from the sweep's lists); the plain and batched forms run
    edm_simplex_sweep then edm_ccm.  With timing on, every launch of the
    timed steps is bracketed by HIP events on the context's stream."""
    ctx.set_form(form)
    fused = form == edm.EDM_FORM_CHOSEN

    def step():
        if fused:
            rs, Es, _ = edm.edm_sweep_ccm(Xd, E_max=E_max, rho=rho, ctx=ctx)
        else:
            rs, Es = edm.edm_simplex_sweep(Xd, E_max=E_max, Tp=1, ctx=ctx)
            edm.edm_ccm(Xd, Es, Tp=0, rho=rho, ctx=ctx)
        return rs, Es

    for _ in range(warmup):
        step()
    ctx.sync()
    torch.cuda.synchronize()
    if timing:
        ctx.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        rs, Es = step()
    ctx.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fam = None
    if timing:
        fam = ctx.timing()
        ctx.set_timing(False)
    return dict(ms_per_step=wall * 1e3 / steps, families=fam, rs=rs.cpu().numpy(),
                Es=Es.cpu().numpy(), rho=rho.cpu().numpy())


def family_work(fam, form, N, L, E_max, E_star):
    """Algorithmic work per step of a kernel family, the unit that bounds it
    and a one-line description."""
    Es = range(1, E_max + 1)
    used = sorted(set(int(e) for e in E_star if e >= 1))
    if fam == "lookup":
        return lookup_bytes(N, L, E_star), "hbm", \
            "k_lookup<K>: 4 L B of target + 4 B rho per pair, 8 m k B of table per (library, E)"
    if fam == "filter_scan":
        return gram_flops(N, L, 1), "mfma", \
            "k_gram<E_lo,E_hi>: BF16 Gram product, 2 E_hi flops per ordered pair per E group"
    if fam == "batched_scan":
        groups = CHOSEN_EXACT if form == "chosen" else EXACT_GROUPS
        ops = scan_ops_grouped(N, L, groups, 1, E_max)
        if form != "chosen":
            ops += scan_ops_grouped(N, L, [(e, e) for e in used], 0)
        return ops, "alu", "k_sweep_multi: exact float32 keys, 3 E_hi + |group| ops per ordered pair"
    if fam == "exact_scan":
        ops = scan_ops_exact(N, L, Es, 1) + scan_ops_exact(N, L, used, 0)
        return ops, "alu", "k_knn: exact float32 keys, 3 E + 1 ops per ordered pair"
    return None, None, None


def kernel_table(fams, steps, form, N, L, E_max, E_star, ceil=None):
    """Per kernel family: time per step, launches, algorithmic work and its
    fraction of the published peak (and of the measured ceiling, if given)."""
    measured = {} if not ceil else {"hbm": ceil["hbm_copy_GBps"] * 1e9,
                                    "mfma": ceil["mfma_bf16_TFLOPs"] * 1e12,
                                    "alu": ceil["valu_fp32_Tops"] * 1e12}
    out = {}
    for fam, (ms, launches) in fams.items():
        if launches == 0:
            continue
        ms_step = ms / steps
        row = {"ms_per_step": ms_step, "launches_per_step": launches / steps}
        work, bound, desc = family_work(fam, form, N, L, E_max, E_star)
        if work is not None:
            peak, unit, scale = PEAK[bound]
            ach = work / (ms_step / 1e3)
            row.update({"bound": bound, "work_per_step": work, "achieved": ach / scale,
                        "peak": peak / scale, "unit": unit, "frac": ach / peak, "kernel": desc})
            if bound in measured:
                row["frac_of_measured_ceiling"] = ach / measured[bound]
        out[fam] = row
    return out


def roofline_of(kt, steps):
    """The dominant family's roofline entry (most time per step)."""
    fam = max(kt, key=lambda f: kt[f]["ms_per_step"])
    r = kt[fam]
    if "bound" not in r:
        return {"family": fam, "bound": None, "achieved": None, "peak": None, "unit": None,
                "frac": None, "traffic": None}
    tr = recorded_traffic(fam)
    traffic = None if tr is None else tr["bytes_per_step"] / r["launches_per_step"]
    return {"family": fam, "kernel": r["kernel"], "bound": r["bound"], "achieved": r["achieved"],
            "peak": r["peak"], "unit": r["unit"], "frac": r["frac"], "traffic": traffic,
            "traffic_source": None if tr is None else tr["source"],
            "avg_launch_ms": r["ms_per_step"] / r["launches_per_step"],
            "work_per_launch": r["work_per_step"] / r["launches_per_step"],
            "frac_of_measured_ceiling": r.get("frac_of_measured_ceiling")}


def parity_subset(group, N, seed=4):
    """16 libraries (4 + 4 sharing two latent drivers, 8 others) and 16
    targets (the driven ones reversed, 8 others), seeded."""
    rng = np.random.default_rng(seed)
    driven = [np.nonzero(group == g)[0][:4] for g in (0, 1)]
    others = rng.choice(np.nonzero(group < 0)[0], size=8, replace=False)
    libs = np.sort(np.r_[driven[0], driven[1], others])
    tgts = np.sort(np.r_[driven[0][::-1], driven[1][::-1],
                         rng.choice(np.setdiff1d(np.arange(N), libs), size=8, replace=False)])
    return libs, tgts


def bench_main(args, torch, edm, synth, wl, name):
    if name == "calcium":
        X, group = synth.calcium_like(seed=wl["seed"], N=wl["N"], L=wl["L"])
        desc = (f"calcium-like {wl['N']} series x L={wl['L']} float32 (20% driven by 20 latent "
                f"logistic maps); simplex E sweep 1..{wl['E_max']} (Tp=1) then full "
                f"{wl['N']}x{wl['N']} CCM (Tp=0) at the targets' E*, k=E+1, self excluded")
    else:
        X, _, _ = synth.logistic_network(seed=wl["seed"], N=wl["N"], L=wl["L"])
        group = None
        desc = (f"logistic-network {wl['N']} series x L={wl['L']} float32; simplex E sweep "
                f"1..{wl['E_max']} (Tp=1) then full {wl['N']}x{wl['N']} CCM (Tp=0), k=E+1, self excluded")
    N, L = X.shape
    E_max = wl["E_max"]
    torch.cuda.set_device(0)
    Xd = torch.from_numpy(X).cuda()
    ctx = edm.Context(device=0)
    rho = torch.empty((N, N), dtype=torch.float32, device="cuda")
    pairs = N * N
    forms = {"plain": [edm.EDM_FORM_PLAIN, edm.EDM_FORM_CHOSEN],
             "all": [edm.EDM_FORM_PLAIN, edm.EDM_FORM_BATCHED, edm.EDM_FORM_CHOSEN],
             "chosen": [edm.EDM_FORM_CHOSEN]}[args.form]
    names = {edm.EDM_FORM_PLAIN: "plain", edm.EDM_FORM_BATCHED: "batched", edm.EDM_FORM_CHOSEN: "chosen"}
    ceil = ctx.ceilings()  # this library's own copy, MFMA and VALU kernels
    res = {}
    for f in forms:
        res[names[f]] = run_form(torch, edm, ctx, Xd, rho, E_max, args.steps, args.warmup, f, True)
    r = res["chosen"]
    kt = kernel_table(r["families"], args.steps, "chosen", N, L, E_max, r["Es"], ceil)
    out = {
        "metric": "CCM pairs/sec at rho err <=1e-5 vs FP64 oracle; chosen vs plain form, 1 GPU",
        "value": pairs / (r["ms_per_step"] / 1e3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "form": "chosen", "series": N, "samples": L,
                   "pairs_per_step": pairs, "parallelism": "single-gpu"},
        "E_star_hist": np.bincount(r["Es"], minlength=E_max + 1)[1:].tolist(),
        "kernels": kt,
        "roofline": roofline_of(kt, args.steps),
        "measured_ceilings": ceil,
    }
    for fname in res:
        if fname == "chosen":
            continue
        p = res[fname]
        same = (np.array_equal(p["rs"].view(np.int32), r["rs"].view(np.int32))
                and np.array_equal(p["Es"], r["Es"])
                and np.array_equal(p["rho"].view(np.int32), r["rho"].view(np.int32)))
        kp = kernel_table(p["families"], args.steps, fname, N, L, E_max, p["Es"], ceil)
        out[fname] = {"value": pairs / (p["ms_per_step"] / 1e3), "ms_per_step": p["ms_per_step"],
                      "kernels": kp, "chosen_speedup": p["ms_per_step"] / r["ms_per_step"],
                      "chosen_bit_identical": bool(same)}
    if "plain" in out:
        out["speedup_vs_plain"] = out["plain"]["chosen_speedup"]

    if not args.no_cpu_baseline:
        cores = args.cores or min(16, os.cpu_count() or 1)
        if group is not None:
            libs, tgts = parity_subset(group, N)
        else:
            rng = np.random.default_rng(wl["seed"])
            libs = np.sort(rng.choice(N, 16, replace=False))
            tgts = np.sort(rng.choice(N, 16, replace=False))
        E_star = r["Es"]
        wall, got = cpu_leg(X, tgts, libs, E_star, E_max, cores)
        sweeps = {t[1]: (t[2], t[3]) for t in got if t[0] == "sweep"}
        rows = {t[1]: (t[2], t[3]) for t in got if t[0] == "row"}
        # sweep parity: rho everywhere, E* equal or a near tie of the oracle's rho
        err_sweep, e_ok, e_diff = 0.0, True, 0
        for s, (ro, eo) in sweeps.items():
            err_sweep = max(err_sweep, float(np.nanmax(np.abs(r["rs"][s].astype(np.float64) - ro))))
            eg = int(r["Es"][s])
            if eg != eo:
                e_diff += 1
                e_ok &= eg >= 1 and abs(ro[eg - 1] - ro[eo - 1]) < 2e-5
        # cross-map rows: every target of the 16 libraries
        err_rows = 0.0
        nan_ok = True
        for i, (ro, _) in rows.items():
            g = r["rho"][i].astype(np.float64)
            nan_ok &= bool(np.array_equal(np.isnan(g), np.isnan(ro)))
            err_rows = max(err_rows, float(np.nanmax(np.abs(g - ro))))
        sub = np.array([[r["rho"][i][j] for j in tgts] for i in libs], dtype=np.float64)
        osub = np.array([[rows[i][0][j] for j in tgts] for i in libs])
        err_sub = float(np.nanmax(np.abs(sub - osub)))
        # tables of the 16 libraries at every E in use, bit for bit (plain form)
        ctx.set_form(edm.EDM_FORM_PLAIN)
        tbl_ok, n_tbl = True, 0
        for i, (_, hashes) in rows.items():
            for E, h in hashes.items():
                idx, _, _ = edm.edm_knn(Xd[i].contiguous(), E, 1, 0, want_dist=False, want_w=False, ctx=ctx)
                gh = hashlib.sha1(idx.cpu().numpy().astype(np.int32).tobytes()).hexdigest()
                tbl_ok &= gh == h
                n_tbl += 1
        ctx.set_form(edm.EDM_FORM_CHOSEN)
        tbl_ok_c = True
        for i, (_, hashes) in list(rows.items())[:4]:
            for E, h in hashes.items():
                idx, _, _ = edm.edm_knn(Xd[i].contiguous(), E, 1, 0, want_dist=False, want_w=False, ctx=ctx)
                tbl_ok_c &= hashlib.sha1(idx.cpu().numpy().astype(np.int32).tobytes()).hexdigest() == h
        ctx.sync()
        frac = len(libs) / N
        out["cpu_baseline"] = {
            "value": pairs * frac / wall, "unit": "pairs/s", "cores": cores,
            "host_cpus": os.cpu_count(), "kind": "oracle",
            "sample": f"{len(tgts)} series' E sweeps 1..{E_max} and {len(libs)} libraries' full CCM rows "
                      f"(x {N} targets at the GPU's E*) = {len(libs)}/{N} of the step; "
                      f"value = {len(libs)} x {N} pairs / wall {wall:.1f} s on {cores} single-threaded workers",
        }
        out["parity"] = {
            "form": "chosen",
            "max_abs_rho_err_sweep": err_sweep,
            "E_star_differs": e_diff,
            "E_star_near_tie_ok": bool(e_ok),
            "max_abs_rho_err_rows": err_rows,
            "rows_pairs": len(libs) * N,
            "max_abs_rho_err_256_subset": err_sub,
            "nan_pattern_equal": bool(nan_ok),
            "tables_bit_exact": bool(tbl_ok and tbl_ok_c),
            "tables_checked": n_tbl,
            "ok": bool(err_sweep <= 1e-5 and err_rows <= 1e-5 and e_ok and nan_ok and tbl_ok and tbl_ok_c),
        }
    ctx.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--form", choices=("plain", "all", "chosen"), default="plain",
                    help="plain: time the plain and the chosen form (default); all: also the "
                         "batched form; chosen: only the chosen form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one device-to-device copy of 256 MiB, whose FETCH_SIZE / "
                         "WRITE_SIZE counters scale the kernels' HBM byte counts")
    ap.add_argument("--cores", type=int, default=0, help="CPU baseline workers (0: min(16, cpus))")
    ap.add_argument("--workload", choices=("calcium", "network", "uneven", "learned", "twokernel"),
                    default="calcium")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(library rows shard across GPUs with no collective, see the design notes)",
              file=sys.stderr)
        return 2

    import torch

    from paper_2105_12301_amd import edm, synth

    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.workload == "uneven":
        out = bench_uneven(args, torch, edm, synth)
    elif args.workload == "learned":
        out = bench_learned(args, torch, edm, synth)
    elif args.workload == "twokernel":
        out = bench_twokernel(args, torch, edm, synth)
    else:
        wl = CALCIUM if args.workload == "calcium" else NETWORK
        out = bench_main(args, torch, edm, synth, wl, args.workload)
    print(json.dumps(out), flush=True)
    _stop_helpers()
    return 0


def _stop_helpers():
    """Stop multiprocessing's resource tracker, which the spawned worker pools
    of the CPU leg start, so that no helper process outlives the benchmark."""
    try:
        import gc
        from multiprocessing import resource_tracker
        gc.collect()  # released pools unregister their semaphores first
        resource_tracker._resource_tracker._stop()
    except Exception:  # private interface: best effort only
        pass


# ------------------------------------------------------- variant workloads --
def _oracle_pairs_task(args):
    x, Lx, Y, Ly, E, cols, Tp = args
    from oracle import edm_oracle as O
    return O.ccm(x[None, :], [Lx], Y, Ly, E, Tp=Tp, tgt_cols=cols)[0]


def _pool_map(fn, tasks, cores):
    import multiprocessing as mp
    pool = mp.get_context("spawn").Pool(cores)
    try:
        t0 = time.perf_counter()
        res = pool.map(fn, tasks, chunksize=1)
        wall = time.perf_counter() - t0
    finally:
        pool.close()
        pool.join()
    return wall, res


def bench_uneven(args, torch, edm, synth):
    """4096 AR(1)-filtered spike-train series, L ~ U{1000..20000}, E ~ U{1..20}
    given per target; all-to-all CCM of the defined pairs (L_target >= L_library).
    Plain: edm_ccm one E at a time.  Plan: autotuned work lists replayed as a
    graph, in the chosen form (matrix-core filter for E >= 5)."""
    from paper_2105_12301_amd import autotune

    X, lens, E = synth.spike_trains(seed=3)
    N = X.shape[0]
    side = torch.cuda.Stream()
    torch.cuda.set_device(0)
    with torch.cuda.stream(side):
        ctx = edm.Context(device=0, stream=side)
        Xd, Ed = torch.from_numpy(X).cuda(), torch.from_numpy(E).cuda()
        rho = torch.empty((N, N), dtype=torch.float32, device="cuda")
        Ls = np.sort(lens)
        pairs = int(sum(N - np.searchsorted(Ls, L, side="left") for L in lens))

        def timed(fn, steps, warmup):
            for _ in range(warmup):
                fn()
            ctx.sync()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record(side)
            for _ in range(steps):
                fn()
            ev[1].record(side)
            ev[1].synchronize()
            return ev[0].elapsed_time(ev[1]) / steps

        ctx.set_form(edm.EDM_FORM_PLAIN)
        ms_plain = timed(lambda: edm.edm_ccm(Xd, Ed, Lx=lens, Ly=lens, rho=rho, ctx=ctx), args.steps, args.warmup)
        ref = rho.clone()
        ctx.set_form(edm.EDM_FORM_CHOSEN)
        t0 = time.perf_counter()
        tune, times = autotune.autotune(Xd, lens, Xd, lens, E, ctx=ctx, use_cache=False)
        t_tune = time.perf_counter() - t0
        plan = edm.CcmPlan(lens, lens, E, X.shape[1], X.shape[1], tune=tune, ctx=ctx)
        ms_plan = timed(lambda: plan.run(Xd, Xd, rho), args.steps, max(1, args.warmup))
        same = bool(torch.equal(ref.view(torch.int32), rho.view(torch.int32)))
        out = {
            "metric": "CCM pairs/sec at rho err <=1e-5 vs FP64 oracle; chosen-form plan vs plain form, 1 GPU",
            "value": pairs / (ms_plan / 1e3), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_plan, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "spike trains 4096 series, L~U{1000..20000}, E~U{1..20} per target, "
                                   "CCM of defined pairs (Tp=0)", "form": "chosen plan (graph)",
                       "defined_pairs": pairs},
            "plain": {"value": pairs / (ms_plain / 1e3), "ms_per_step": ms_plain},
            "speedup_vs_plain": ms_plain / ms_plan,
            "bit_identical_to_plain": same,
            "autotune": {"chosen": tune.as_dict(), "seconds": t_tune, "candidates_ms_on_sample": times},
        }
        plan.close()
        if not args.no_cpu_baseline:
            # oracle on the shortest, the median and the longest library x 64 defined targets
            rng = np.random.default_rng(0)
            order = np.argsort(lens, kind="stable")
            libs = [order[0], order[1], order[N // 2], order[-1]]
            tasks = []
            for i in libs:
                cols = np.nonzero(lens >= lens[i])[0]
                cols = np.sort(rng.choice(cols, size=min(64, cols.size), replace=False))
                tasks.append((X[i, :lens[i]], int(lens[i]), X, lens, E, cols, 0))
            cores = min(args.cores or min(16, os.cpu_count() or 1), len(tasks))
            wall, res = _pool_map(_oracle_pairs_task, tasks, cores)
            g = rho.cpu().numpy()
            err = max(float(np.nanmax(np.abs(g[i, t[5]] - r))) for i, t, r in zip(libs, tasks, res))
            npairs = sum(len(t[5]) for t in tasks)
            out["cpu_baseline"] = {"value": npairs / wall, "unit": "pairs/s", "cores": cores,
                                   "host_cpus": os.cpu_count(), "kind": "oracle",
                                   "sample": f"{npairs} pairs: the 2 shortest, the median and the longest "
                                             "library x 64 random defined targets"}
            out["parity"] = {"max_abs_rho_err": err, "ok": err <= 1e-5}
        ctx.close()
    return out


def bench_learned(args, torch, edm, synth):
    """Learned E surrogate: train on 50000 labelled series (logistic, Lorenz x,
    AR(2); L = 1500), then one GPU's share of a 100000-series CCM (library rows
    0..1023 vs all targets).  E selection by the full sweep vs by the network
    with top-3 verification and the confidence fallback; the sweep judges the
    rho lost."""
    from paper_2105_12301_amd.surrogate import Surrogate

    torch.cuda.set_device(0)
    ctx = edm.Context(device=0, form=edm.EDM_FORM_CHOSEN)
    Xtr, _ = synth.surrogate_mix(seed=5, N=50000, L=1500)
    Xtr_d = torch.from_numpy(Xtr).cuda()
    t0 = time.perf_counter()
    rs_tr, Etr = edm.edm_simplex_sweep(Xtr_d, E_max=20, Tp=1, ctx=ctx)
    ctx.sync()
    t_label = time.perf_counter() - t0
    sur = Surrogate(C=64, seed=0, ctx=ctx)
    t0 = time.perf_counter()
    hist = sur.train(Xtr_d[:45000], Etr[:45000], epochs=8, batch=256, lr=2e-3)
    ctx.sync()
    t_train = time.perf_counter() - t0
    val_acc = sur.accuracy(Xtr_d[45000:].contiguous(), Etr[45000:].contiguous())
    min_conf = sur.calibrate(Xtr_d[45000:].contiguous(), rs_tr[45000:].contiguous(), m_top=3)
    del Xtr_d
    X, _ = synth.surrogate_mix(seed=6, N=100000, L=1500)
    Xd = torch.from_numpy(X).cuda()
    nlib = 1024
    lib = Xd[:nlib]
    rho = torch.empty((nlib, X.shape[0]), dtype=torch.float32, device="cuda")
    nfb = {}

    def run_sweep():
        rs, Es = edm.edm_simplex_sweep(Xd, E_max=20, Tp=1, ctx=ctx)
        edm.edm_ccm(lib, Es, Y=Xd, rho=rho, ctx=ctx)
        return rs, Es

    def run_net(mc):
        def f():
            r, Es, n = sur.select_E(Xd, m_top=3, min_conf=mc)
            nfb[mc] = n
            edm.edm_ccm(lib, Es, Y=Xd, rho=rho, ctx=ctx)
            return r, Es
        return f

    def timed(fn):
        fn()
        ctx.sync()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            res = fn()
        ctx.sync()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / args.steps, res

    ms_sweep, (rs, Es) = timed(run_sweep)
    rs_h, Es_h = rs.cpu().numpy().astype(np.float64), Es.cpu().numpy()
    best = np.nanmax(rs_h, axis=1)
    sel = {}
    for mc in (0.0, min_conf):
        ms, (rn, En) = timed(run_net(mc))
        En_h = En.cpu().numpy()
        got = rs_h[np.arange(len(En_h)), En_h - 1]
        loss = best - got
        sel[mc] = {"ms_per_step": ms, "min_conf": mc, "n_fallback": int(nfb[mc]),
                   "E_equal_to_sweep": float(np.mean(En_h == Es_h)),
                   "mean_rho_loss": float(np.mean(loss)), "p99_rho_loss": float(np.quantile(loss, 0.99)),
                   "max_rho_loss": float(np.max(loss)), "speedup_vs_sweep": ms_sweep / ms}
    main_sel = sel[min_conf]
    pairs = nlib * X.shape[0]
    out = {
        "metric": "CCM pairs/sec (E selection + CCM); learned E surrogate vs full simplex sweep, 1 GPU",
        "value": pairs / (main_sel["ms_per_step"] / 1e3), "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": main_sel["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "surrogate mix (logistic, Lorenz x, AR(2)), L=1500: train 50000 "
                               "series, then library rows 0..1023 x 100000 targets",
                   "form": "chosen + learned E (top-3 verified, confidence fallback)"},
        "sweep_based": {"value": pairs / (ms_sweep / 1e3), "ms_per_step": ms_sweep},
        "speedup_vs_sweep": main_sel["speedup_vs_sweep"],
        "training": {"label_s": t_label, "train_s": t_train, "epochs": len(hist),
                     "final_loss": hist[-1][0], "val_top1": val_acc},
        "selection_with_fallback": main_sel,
        "selection_without_fallback": sel[0.0],
    }
    if not args.no_cpu_baseline:
        # oracle rho of 16 libraries x 16 targets at the network-selected E
        rng = np.random.default_rng(6)
        libs = np.arange(16)
        tgts = np.sort(rng.choice(X.shape[0], 16, replace=False))
        sur.select_E(Xd, m_top=3, min_conf=min_conf)
        r_net, E_net, _ = sur.select_E(Xd, m_top=3, min_conf=min_conf)
        E_net_h = E_net.cpu().numpy()
        edm.edm_ccm(lib, E_net, Y=Xd, rho=rho, ctx=ctx)
        ctx.sync()
        g = rho.cpu().numpy()[np.ix_(libs, tgts)]
        tasks = [(X[i], 1500, X[tgts], np.full(16, 1500), E_net_h[tgts], np.arange(16), 0) for i in libs]
        cores = min(args.cores or min(16, os.cpu_count() or 1), len(tasks))
        wall, res = _pool_map(_oracle_pairs_task, tasks, cores)
        err = float(np.nanmax(np.abs(g - np.array(res))))
        out["cpu_baseline"] = {"value": 256 / wall, "unit": "pairs/s", "cores": cores,
                               "host_cpus": os.cpu_count(), "kind": "oracle",
                               "sample": "256 pairs: libraries 0..15 x 16 random targets at the "
                                         "network-selected E"}
        out["parity"] = {"max_abs_rho_err": err, "ok": err <= 1e-5}
    ctx.close()
    return out


def bench_twokernel(args, torch, edm, synth):
    """The paper's two-kernel kNN (distance matrix in HBM, then per-row top-k)
    against the fused scan.  Part 1, the paper's kNN breakdown: one series of
    L = 10^4 samples, E = 1..20, Tp = 0, k = E+1, one table per E (HIP-event
    time per kernel family, median of the timed repetitions).  Part 2, the
    calcium-like 10000 x 2000 step (sweep + full cross map) in the two-kernel
    form next to the plain fused form."""
    torch.cuda.set_device(0)
    ctx = edm.Context(device=0)
    X = synth.logistic_network(seed=7, N=4, L=10000)[0]
    x = torch.from_numpy(X[0].copy()).cuda()
    L = X.shape[1]
    reps = max(1, args.steps)
    rows = []
    for E in range(1, 21):
        m = L - (E - 1)
        rec = {"E": E, "m": m}
        for fname, form in (("two_kernel", edm.EDM_FORM_TWO_KERNEL), ("fused", edm.EDM_FORM_PLAIN),
                            ("chosen", edm.EDM_FORM_CHOSEN)):
            ctx.set_form(form)
            for _ in range(max(1, args.warmup)):
                edm.edm_knn(x, E, 1, 0, want_dist=False, ctx=ctx)
            ctx.sync()
            per = []
            for _ in range(reps):
                ctx.set_timing(True)
                edm.edm_knn(x, E, 1, 0, want_dist=False, ctx=ctx)
                per.append(ctx.timing())
                ctx.set_timing(False)
            fams = {f for t in per for f, (ms, n) in t.items() if n}
            rec[fname] = {f: float(np.median([t[f][0] for t in per])) for f in fams}
        d_ms = rec["two_kernel"]["distances"]
        t_ms = rec["two_kernel"]["row_topk"]
        rec["distances_GBps_written"] = 4.0 * m * m / (d_ms / 1e3) / 1e9
        rec["distances_Tops"] = 3.0 * E * m * m / (d_ms / 1e3) / 1e12
        rec["row_topk_GBps_read"] = 4.0 * m * m / (t_ms / 1e3) / 1e9
        rec["fused_over_two_kernel"] = (d_ms + t_ms) / sum(rec["fused"].values())
        rows.append(rec)
    ctx.set_form(edm.EDM_FORM_PLAIN)
    out = {"metric": "kNN table time per E, two-kernel (paper) vs fused, 1 GPU",
           "unit": "ms", "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "one logistic-network series, L=10000, E=1..20, Tp=0, k=E+1"},
           "per_E": rows}
    # Part 2: the headline step in the two-kernel form.
    wl = CALCIUM
    Xc, _ = synth.calcium_like(seed=wl["seed"], N=wl["N"], L=wl["L"])
    Xd = torch.from_numpy(Xc).cuda()
    N = Xc.shape[0]
    rho = torch.empty((N, N), dtype=torch.float32, device="cuda")
    steps = max(1, min(args.steps, 2))
    r2 = run_form(torch, edm, ctx, Xd, rho, wl["E_max"], steps, 1, edm.EDM_FORM_TWO_KERNEL, True)
    r1 = run_form(torch, edm, ctx, Xd, rho, wl["E_max"], steps, 1, edm.EDM_FORM_PLAIN, True)
    same = (np.array_equal(r1["rs"].view(np.int32), r2["rs"].view(np.int32))
            and np.array_equal(r1["Es"], r2["Es"])
            and np.array_equal(r1["rho"].view(np.int32), r2["rho"].view(np.int32)))
    fam2 = {f: ms / steps for f, (ms, n) in r2["families"].items() if n}
    fam1 = {f: ms / steps for f, (ms, n) in r1["families"].items() if n}
    m_sum = sum(_m(wl["L"], E, 1) ** 2 for E in range(1, 21)) + \
        sum(_m(wl["L"], E, 0) ** 2 for E in sorted(set(int(e) for e in r2["Es"] if e >= 1)))
    out["calcium_step"] = {
        "workload": "calcium-like 10000 x 2000: E sweep 1..20 + full CCM",
        "two_kernel_ms_per_step": r2["ms_per_step"], "plain_fused_ms_per_step": r1["ms_per_step"],
        "two_kernel_families_ms": fam2, "plain_families_ms": fam1,
        "distance_matrix_bytes_per_step": 4.0 * N * m_sum,
        "distances_GBps_written": 4.0 * N * m_sum / (fam2["distances"] / 1e3) / 1e9,
        "row_topk_GBps_read": 4.0 * N * m_sum / (fam2["row_topk"] / 1e3) / 1e9,
        "bit_identical": bool(same), "steps": steps}
    ctx.close()
    return out


if __name__ == "__main__":
    sys.exit(main())
