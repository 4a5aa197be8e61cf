"""Benchmark: one leapfrog step of the tree-code per step (sort, build,
moments, walk + force, kicks and drift) on one MI355X.

Prints one JSON line.  `value` is tree-walk interactions (particle-particle +
particle-cell) per second of whole-step wall time; the walk kernel's own
rate and its Tflops under the paper's convention (Sec. VI.A: 23 flops per
particle-particle and 65 per particle-cell interaction) are reported beside
it, with the walk's fraction of the FP32 vector peak.  The CPU baseline is
the oracle (FP64 C tree code) timed on a bounded sample of the same
workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FLOPS_PP = 23
FLOPS_PC = 65
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector peak (256 CUs x 2.4 GHz x 256 flop/clk)
WALK_SOURCES = [os.path.join(ROOT, "paper_1412_0659_amd", "csrc", f)
                for f in ("walk.hip", "walk_common.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "walk_disk_halo_13m_traffic.json")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "walk_valu_counters_disk_halo_13m.json")
VJP_SOURCES = [os.path.join(ROOT, "paper_1412_0659_amd", "csrc", f)
               for f in ("walk_vjp.hip", "walk_common.h")]


def paper_flops(n_pp, n_pc):
    """Flops of a walk under the paper's convention (Sec. VI.A)."""
    return FLOPS_PP * float(n_pp) + FLOPS_PC * float(n_pc)


def walk_source_hash(paths=None):
    """Hash of a kernel's sources (default: the walk's evaluation and traversal)."""
    h = hashlib.sha256()
    for path in (WALK_SOURCES if paths is None else paths):
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_counters():
    """Per-dispatch VALU counters of the walk kernels and the force VJP from
    the committed rocprofv3 summary, each kept only if taken on the current
    source of its kernel (None otherwise)."""
    try:
        with open(COUNTERS_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    ok_walk = t.get("walk_source_sha256_16") == walk_source_hash()
    ok_vjp = t.get("vjp_source_sha256_16") == walk_source_hash(VJP_SOURCES)
    out = {}
    for name, c in t.get("kernels", {}).items():
        if (name.startswith("k_walk_vjp") and ok_vjp) or (not name.startswith("k_walk_vjp")
                                                          and ok_walk):
            out[name] = c
    return out or None


def counter_flops(c):
    """FP32 + FP16 VALU flops of one dispatch from its counters: the
    hardware's own FLOPS counts (transcendentals included; they count per
    wave instruction, so x 64 lanes), and the count derived from the
    instruction classes (FMA 2, add / mul / rsq 1 per lane)."""
    hw = 64.0 * sum(c.get(k, 0.0) for k in (
        "SQ_INSTS_VALU_FLOPS_FP32", "SQ_INSTS_VALU_FLOPS_FP32_TRANS",
        "SQ_INSTS_VALU_FLOPS_FP16", "SQ_INSTS_VALU_FLOPS_FP16_TRANS"))
    ins = 64.0 * (2 * c.get("SQ_INSTS_VALU_FMA_F32", 0.0) + c.get("SQ_INSTS_VALU_MUL_F32", 0.0)
                  + c.get("SQ_INSTS_VALU_ADD_F32", 0.0) + c.get("SQ_INSTS_VALU_TRANS_F32", 0.0))
    return hw, ins


def pmc_rows(db):
    """Every dispatch of a rocprofv3 --pmc output database (sqlite) in launch
    order: [{"kernel": name, "ms": duration, counter: value, ...}]."""
    import sqlite3
    con = sqlite3.connect(db)
    q = ("select ks.display_name, kd.id, ip.name, sum(pe.value), kd.end - kd.start "
         "from rocpd_pmc_event pe join rocpd_info_pmc ip on pe.pmc_id = ip.id "
         "join rocpd_kernel_dispatch kd on pe.event_id = kd.event_id "
         "join rocpd_info_kernel_symbol ks on kd.kernel_id = ks.id group by kd.id, ip.name "
         "order by kd.id")
    rows = {}
    for name, did, cname, val, d in con.execute(q):
        r = rows.setdefault(did, {"kernel": name, "ms": d / 1e6})
        r[cname] = val
    con.close()
    return [rows[k] for k in sorted(rows)]


def pmc_dispatches(paths):
    """Counter values of every dispatch in rocprofv3 --pmc output databases
    (sqlite): {kernel: [{counter: value, "ms": duration}, ...]}."""
    from collections import defaultdict
    out = defaultdict(list)
    for db in paths:
        for r in pmc_rows(db):
            r = dict(r)
            out[r.pop("kernel")].append(r)
    return out


def build_phase_counters(db, counter, build_index=1):
    """Sum of one counter over the kernels of each phase of one tree build in
    a --pmc database: the build_index-th build (a build starts at a
    k_bbox_partial dispatch); sort = through k_gather, build = up to the
    first moments kernel, moments = the k_moments_ kernels."""
    rows = pmc_rows(db)
    starts = [i for i, r in enumerate(rows) if "k_bbox_partial" in r["kernel"]]
    i = starts[build_index]
    out = {"sort": 0.0, "build": 0.0, "moments": 0.0}
    phase = "sort"
    kernels = {k: [] for k in out}
    for r in rows[i:]:
        name = r["kernel"]
        if phase == "moments" and "k_moments_" not in name:
            break
        if "k_moments_" in name:
            phase = "moments"
        out[phase] += r.get(counter, 0.0)
        short = name.replace("void ", "").split("(")[0].replace("bh::", "")
        if short not in kernels[phase]:
            kernels[phase].append(short)
        if "k_gather" in name:
            phase = "build"
    return out, kernels


def write_build_traffic(out_path, fetch_db, write_db, bench_json, command):
    """HBM bytes of the tree-build phases of the first leapfrog step's
    rebuild: FETCH_SIZE and WRITE_SIZE (KiB) scaled by the copy calibration
    of the committed walk traffic file, against the algorithmic bytes of
    hbm_phases for the tree of the bench line in bench_json."""
    with open(TRAFFIC_FILE) as f:
        cal = json.load(f)["copy_calibration"]
    ff, wf = cal["fetch_factor"], cal["write_factor"]
    fetch, kernels = build_phase_counters(fetch_db, "FETCH_SIZE")
    write, _ = build_phase_counters(write_db, "WRITE_SIZE")
    with open(bench_json) as f:
        line = json.loads([l for l in f if l.startswith("{")][-1])
    n, tree, ms = line["config"]["n"], line["tree"], line["ms_phase"]
    alg = hbm_phases(n, tree["cells"], ms["sort"], ms["moments"], ms_build=ms["build"],
                     depth=tree["depth"])
    hdr = [f"# HBM bytes of the tree rebuild of the first leapfrog step at {line['config']['workload']}"
           f" ({n} particles, {tree['cells']} cells),",
           f"# from rocprofv3 counters: FETCH_SIZE x {ff:.3f} + WRITE_SIZE x {wf:.3f} (the factors a plain"
           " 1 GiB device copy reads for the same counters), summed over each phase's kernels of"
           " that build (particles already nearly in key order).",
           "# ms: the bench line's mean phase time (events, no profiler); GB/s = counted bytes / ms.",
           f"# commands: {command}",
           "#",
           f"{'phase':9s} {'fetch_MB':>9s} {'write_MB':>9s} {'total_MB':>9s} {'algorithmic_MB':>15s}"
           f" {'ratio':>6s} {'ms':>7s} {'GB/s':>8s}  kernels"]
    rows = []
    for ph in ("sort", "build", "moments"):
        f_b = fetch[ph] * 1024.0 * ff
        w_b = write[ph] * 1024.0 * wf
        a_b = alg[ph]["bytes"] if ph in alg else None
        t = ms[ph]
        rows.append(f"{ph:9s} {f_b / 1e6:9.1f} {w_b / 1e6:9.1f} {(f_b + w_b) / 1e6:9.1f} "
                    f"{(a_b / 1e6 if a_b else float('nan')):15.1f} "
                    f"{((f_b + w_b) / a_b if a_b else float('nan')):6.2f} {t:7.3f} "
                    f"{(f_b + w_b) / (t * 1e-3) / 1e9:8.1f}  {', '.join(kernels[ph])}")
    foot = ["#",
            "# algorithmic bytes (hbm_phases): sort 376 B per particle (box 12, keys 24, 8 radix",
            "# passes x 32, gather 84); build: the keys read once per splitting level plus 40 B per",
            "# cell and 12 B per particle for the groups (what a per-level scan would move; the",
            "# build's binary searches over cell ranges read less); moments: 16 B per particle +",
            "# 260 B per cell (topology 20, FP64 M, S, Q written 80 and read by the parent 80, walk",
            "# records 80)."]
    text = "\n".join(hdr + rows + foot) + "\n"
    with open(out_path, "w") as f:
        f.write(text)
    return text


def pmc_summary(paths, min_frac=0.0):
    """Mean counter value per dispatch and mean duration of every kernel in
    rocprofv3 --pmc output databases; with min_frac only the dispatches at
    least that fraction of the kernel's longest one (the full-size workload
    among smaller ones): {kernel: {counter: value}}."""
    out = {}
    for name, rows in pmc_dispatches(paths).items():
        longest = max(r["ms"] for r in rows)
        sel = [r for r in rows if r["ms"] >= min_frac * longest]
        keys = sorted({k for r in sel for k in r if k != "ms"})
        row = {k: sum(r[k] for r in sel if k in r) / max(1, sum(1 for r in sel if k in r))
               for k in keys}
        row["dispatches"] = len(sel)
        row["mean_ms"] = sum(r["ms"] for r in sel) / len(sel)
        out[name] = row
    return out


def load_traffic():
    """HBM bytes per walk launch from the committed rocprofv3 counter summary,
    or None if absent or taken on a different walk kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("walk_source_sha256_16") != walk_source_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_model():
    """Host CPU model name and logical CPU count."""
    name = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": name, "os_cpu_count": os.cpu_count()}


def oracle_anchors(anchors, nanchor=256):
    """The oracle's FP64 direct sum at the first `nanchor` sampled targets of
    each GPU error measurement: it checks the GPU's FP64 direct sum (the
    reference of the full-sample errors) and the walks' errors directly."""
    import numpy as np

    from oracle import oracle as O
    out = {}
    for a in anchors:
        idx = a["idx"][:nanchor]
        t0 = time.perf_counter()
        oa, op = O.direct(a["pos"], a["mass"], np.float32(a["eps"]), targets=idx)
        dt = time.perf_counter() - t0
        r = {"targets": int(len(idx)), "oracle_direct_s": dt,
             "gpu_direct_vs_oracle_max_rel": float(np.max(_rel(a["ref_acc"][:nanchor], oa)))}
        for k, acc in a["walks"].items():
            e = _rel(acc[:nanchor], oa)
            r[k + "_err_acc_median"] = float(np.median(e))
            r[k + "_err_acc_p99"] = float(np.percentile(e, 99))
        out[a["name"]] = r
    return out


def cpu_baseline(snap, theta, eps, budget_s=12.0):
    """Time the oracle's tree walk over a seeded sample of groups."""
    import numpy as np

    from oracle import oracle as O
    t0 = time.perf_counter()
    tree = O.build_tree(snap.pos, snap.mass)
    t_build = time.perf_counter() - t0
    rng = np.random.default_rng(1234)
    order = rng.permutation(tree.ngroups)
    done, inter, walk_s, k = 0, 0, 0.0, 64
    while done < len(order) and walk_s < budget_s:
        sel = order[done:done + k]
        t1 = time.perf_counter()
        _, _, npp, npc = O.walk(tree, theta, eps, groups=sel)
        walk_s += time.perf_counter() - t1
        inter += int(((npp[sel] + npc[sel]) * tree.gcnt[sel]).sum())
        done += len(sel)
        k = min(4 * k, 4096)
    targets = int(tree.gcnt[order[:done]].sum())
    return {
        "value": inter / walk_s, "unit": "interactions/s", "cores": O.num_threads(),
        "kind": "oracle", "cpu": cpu_model(),
        "sample": (f"FP64 oracle walk of {done} random groups ({targets} targets) of the "
                   f"{tree.n}-particle tree, theta={theta}, eps={eps}; {walk_s:.1f} s of walk; "
                   f"oracle tree build over all particles took {t_build:.1f} s (not in value)"),
    }


def cpu_configs(anchors=None, walk_budget_s=3.0):
    """The oracle on the other workloads, on this host: the 16k Plummer sphere
    (full tree force at theta 0.3 / 0.5 / 0.7 and the full O(N^2) direct sum,
    tree-vs-direct error per theta), the 1M disk + halo (tree build and a
    seeded sample of its group walks), and the 4M direct sum at sampled
    targets (taken from the error anchors when given)."""
    import numpy as np

    from oracle import oracle as O
    from workloads import ics
    out = {}
    w = ics.WORKLOADS["plummer_16k"]
    s = ics.make("plummer_16k")
    t0 = time.perf_counter()
    tree = O.build_tree(s.pos, s.mass)
    t_build = time.perf_counter() - t0
    eps32 = float(np.float32(w["eps"]))
    t0 = time.perf_counter()
    da, dp = O.direct(s.pos, s.mass, eps32)
    t_direct = time.perf_counter() - t0
    per_theta = {}
    for theta in (0.3, 0.5, 0.7):
        t0 = time.perf_counter()
        acc, pot, npp, npc = O.walk(tree, theta, w["eps"])
        dt = time.perf_counter() - t0
        inter = int(((npp + npc) * tree.gcnt).sum())
        e = _rel(acc, da)
        per_theta[str(theta)] = {"walk_s": dt, "interactions_per_s": inter / dt,
                                 "err_acc_median": float(np.median(e)),
                                 "err_acc_p99": float(np.percentile(e, 99))}
    out["plummer_16k"] = {
        "n": s.n, "eps": w["eps"], "tree_build_s": t_build, "tree": per_theta,
        "direct_s": t_direct, "direct_pairs_per_s": float(s.n) * s.n / t_direct,
        "note": "full FP64 oracle tree force per theta and full FP64 direct sum; errors of "
                "the oracle tree against the oracle direct sum"}
    w = ics.WORKLOADS["disk_halo_1m"]
    s = ics.make("disk_halo_1m")
    t0 = time.perf_counter()
    tree = O.build_tree(s.pos, s.mass)
    t_build = time.perf_counter() - t0
    order = np.random.default_rng(4321).permutation(tree.ngroups)
    done, inter, walk_s, k = 0, 0, 0.0, 64
    while done < len(order) and walk_s < walk_budget_s:
        sel = order[done:done + k]
        t1 = time.perf_counter()
        _, _, npp, npc = O.walk(tree, w["theta"], w["eps"], groups=sel)
        walk_s += time.perf_counter() - t1
        inter += int(((npp[sel] + npc[sel]) * tree.gcnt[sel]).sum())
        done += len(sel)
        k = min(4 * k, 4096)
    targets = int(tree.gcnt[order[:done]].sum())
    rate = inter / walk_s
    out["disk_halo_1m"] = {
        "n": s.n, "theta": w["theta"], "eps": w["eps"], "tree_build_s": t_build,
        "sample": f"{done} random groups ({targets} targets), {walk_s:.1f} s of walk",
        "interactions_per_s": rate,
        "full_walk_s_estimated": inter / targets * s.n / rate}
    for a in anchors or []:
        if a["name"].startswith("disk_halo_4m"):
            idx = a["idx"][:256]
            t0 = time.perf_counter()
            O.direct(a["pos"], a["mass"], np.float32(a["eps"]), targets=idx)
            dt = time.perf_counter() - t0
            n = len(a["mass"])
            out["disk_halo_4m"] = {
                "n": n, "direct_targets": int(len(idx)), "direct_s": dt,
                "direct_pairs_per_s": float(n) * len(idx) / dt,
                "direct_65536_targets_s_estimated": dt * 65536 / len(idx)}
    return out


def hbm_phases(n, ncells, ms_sort, ms_moments, pos_fp64=False, ms_build=None, depth=None):
    """Algorithmic HBM bytes of the tree-build phases and the rate they imply.

    Per particle, sort phase: box 12 B read; keys 12 B read + 12 B written
    (u64 key, u32 index); 8 radix passes of 8 B read (digit count) + 12 B read
    + 12 B written (scatter); gather 4 B index + 32 B state read, 32 B state +
    16 B (x, y, z, m) record written (+48 B with the FP64 master).
    Moments: 16 B per particle
    read plus, per cell, 20 B of topology read (nchild, first, count, key
    prefix), 80 B of FP64 moments (M, S, Q) written and read back by the
    parent's pass and 80 B of walk records written.
    Build (with ms_build and depth): 8 B of keys per particle per splitting
    level, 36 B written and 4 B read per cell, 12 B per particle for the groups."""
    gather = 4 + 32 + 32 + 16 + (48 if pos_fp64 else 0)
    sort_b = n * (12 + 24 + 8 * 32 + gather)
    mom_b = n * 16 + ncells * (20 + 80 + 80 + 80)
    out = {"sort": {"bytes": sort_b, "ms": ms_sort},
           "moments": {"bytes": mom_b, "ms": ms_moments}}
    if ms_build is not None and depth is not None:
        # octree + groups: the keys read once per level that splits cells
        # (levels 0 .. depth - 1), 36 B written per cell, the group pass
        # 4 B read per cell and 12 B per particle (flags, scan, begin)
        out["build"] = {"bytes": n * 8 * int(depth) + ncells * (36 + 4) + n * 12,
                        "ms": ms_build}
    for v in out.values():
        v["GBps"] = v["bytes"] / (v["ms"] * 1e-3) / 1e9 if v["ms"] > 0 else None
    return out


def _rel(a, ref):
    import numpy as np
    if a.ndim == 1:
        return np.abs(a - ref) / np.abs(ref)
    return np.sqrt(((a - ref) ** 2).sum(1) / (ref ** 2).sum(1))


def _timed_force(tree, theta, eps, reps):
    """Force `reps` times after one warm-up; mean walk-kernel ms and the last
    accelerations / potentials (caller order, float64 numpy)."""
    tree.force(theta, eps)
    tree.sync()
    ms = []
    for _ in range(reps):
        acc, pot = tree.force(theta, eps)
        ms.append(tree.stats()["ms_walk"])
    st = tree.stats()
    return (sum(ms) / len(ms), acc.double().cpu().numpy(), pot.double().cpu().numpy(), st)


def precision(snap, theta, eps, nsample=65536, seed=40, reps=3, log=print, ref=None):
    """Plain FP32 walk vs the FP16 far-field walk on the same particles: walk
    time and force error against the GPU's FP64 direct sum at a seeded
    uniform subsample of targets (ref: that direct sum, if already taken)."""
    import numpy as np
    import torch

    import paper_1412_0659_amd as bh
    from workloads import ics
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(snap.pos).to(dev)
    mass = torch.from_numpy(snap.mass).to(dev)
    idx = ics.subsample(snap.n, nsample, seed)
    tg = torch.from_numpy(idx.astype(np.int64)).to(dev)
    out = {"theta": theta, "eps": eps,
           "sample": f"{len(idx)} targets, seeded uniform subsample (seed {seed}) of "
                     f"{snap.n}; reference: FP64 direct sum on the GPU (tree_direct)"}
    walks = {}
    for name, f16 in (("fp32", False), ("fp16_far", True)):
        tree = bh.Tree(snap.n, far_fp16=f16)
        tree.build(pos, mass)
        if ref is None:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ra, rp = tree.direct(tg, eps)
            tree.sync()
            out["direct_s"] = time.perf_counter() - t0
            ref = (ra.cpu().numpy(), rp.cpu().numpy())
        ms, acc, pot, st = _timed_force(tree, theta, eps, reps)
        tree.close()
        ea = _rel(acc[idx], ref[0])
        ep = _rel(pot[idx], ref[1])
        walks[name] = acc[idx]
        out[name] = {"walk_ms": ms, "err_acc_median": float(np.median(ea)),
                     "err_acc_p99": float(np.percentile(ea, 99)),
                     "err_pot_median": float(np.median(ep)),
                     "n_pp": st["n_pp"], "n_pc": st["n_pc"],
                     "tflops_walk": paper_flops(st["n_pp"], st["n_pc"]) / (ms * 1e-3) / 1e12}
        log(f"[bench] precision {name}: walk {ms:.2f} ms, acc err median "
            f"{out[name]['err_acc_median']:.2e} p99 {out[name]['err_acc_p99']:.2e}")
    out["speedup_walk_fp16_far"] = out["fp32"]["walk_ms"] / out["fp16_far"]["walk_ms"]
    for name in ("fp32", "fp16_far"):
        out[name]["frac_fp32_peak"] = out[name]["tflops_walk"] / PEAK_FP32_TFLOPS
    out["_ref"] = ref
    out["_anchor"] = {"pos": snap.pos, "mass": snap.mass, "eps": eps, "idx": idx,
                      "ref_acc": ref[0], "walks": walks}
    return out


def paired_sets(snap, theta, eps, ref, idx, base_ms, caps=(32, 48, 64), reps=3, log=print):
    """Paired target sets (pair_groups = cap: sibling groups of together at
    most cap particles walked as one): walk time, interactions and force
    error against the precision leg's FP64 direct sum at the same targets;
    base_ms is the plain FP32 walk's time (pair_groups = 0)."""
    import numpy as np
    import torch

    import paper_1412_0659_amd as bh
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(snap.pos).to(dev)
    mass = torch.from_numpy(snap.mass).to(dev)
    rows = []
    for cap in caps:
        tree = bh.Tree(snap.n, pair_groups=cap)
        tree.build(pos, mass)
        ms, acc, pot, st = _timed_force(tree, theta, eps, reps)
        tree.close()
        ea = _rel(acc[idx], ref[0])
        rows.append({"pair_groups": cap, "walk_ms": ms, "speedup_vs_groups": base_ms / ms,
                     "target_sets": st["ngroups"],
                     "pp_per_particle": st["n_pp"] / snap.n, "pc_per_particle": st["n_pc"] / snap.n,
                     "err_acc_median": float(np.median(ea)),
                     "err_acc_p99": float(np.percentile(ea, 99))})
        log(f"[bench] paired target sets <= {cap}: walk {ms:.2f} ms ({base_ms / ms:.3f}x)")
    return {"note": "sibling groups of together <= pair_groups particles walked as one target "
                    "set (bh_params.pair_groups); the default walk (pair_groups = 0) is the "
                    "headline", "rows": rows}


def precision_sweep(name="disk_halo_4m", thetas=(0.3, 0.4, 0.6), log=print):
    """The precision form's table: FP32 and FP16 far-field walks at several
    opening angles, errors against one FP64 direct sum."""
    from workloads import ics
    w = ics.WORKLOADS[name]
    snap = ics.make(name)
    rows, ref, anchor = [], None, None
    for th in thetas:
        r = precision(snap, th, w["eps"], log=log, ref=ref)
        ref = r.pop("_ref")
        a = r.pop("_anchor")
        if abs(th - w["theta"]) < 1e-9:
            anchor = a
        rows.append(r)
    return {"workload": name, "n": snap.n, "eps": w["eps"], "rows": rows, "_anchor": anchor}


def param_sweep(name="disk_halo_4m", thetas=(0.3, 0.4, 0.5, 0.6, 0.8),
                leaf_crit=((16, 64), (8, 64), (32, 64), (16, 32)), reps=2, log=print):
    """Walk cost against the opening angle (the tree-code's cost grows as
    theta^-3) and against the leaf and group sizes, on one model."""
    import torch

    import paper_1412_0659_amd as bh
    from workloads import ics
    w = ics.WORKLOADS[name]
    snap = ics.make(name)
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(snap.pos).to(dev)
    mass = torch.from_numpy(snap.mass).to(dev)
    rows = []
    for nleaf, ncrit in leaf_crit:
        tree = bh.Tree(snap.n, nleaf=nleaf, ncrit=ncrit)
        tree.build(pos, mass)
        st0 = tree.stats()
        for th in (thetas if (nleaf, ncrit) == (16, 64) else (w["theta"],)):
            ms, _, _, st = _timed_force(tree, th, w["eps"], reps)
            inter = st["n_pp"] + st["n_pc"]
            rows.append({"nleaf": nleaf, "ncrit": ncrit, "theta": th, "walk_ms": ms,
                         "pp_per_particle": st["n_pp"] / snap.n,
                         "pc_per_particle": st["n_pc"] / snap.n,
                         "interactions_per_s": inter / (ms * 1e-3),
                         "tflops": paper_flops(st["n_pp"], st["n_pc"]) / (ms * 1e-3) / 1e12,
                         "cells": st0["ncells"], "groups": st0["ngroups"],
                         "build_ms": st0["ms_sort"] + st0["ms_build"] + st0["ms_moments"]})
            log(f"[bench] nleaf {nleaf} ncrit {ncrit} theta {th}: walk {ms:.2f} ms")
        tree.close()
    return {"workload": name, "n": snap.n, "eps": w["eps"], "rows": rows}


def adjoint(name="disk_halo_1m_adjoint", log=print, pair_groups=0):
    """The differentiation workload: K KDK steps forward with checkpoints,
    surface-density loss, reverse sweep; forward and backward wall time
    (pair_groups: the context's paired target sets, 0 = groups)."""
    import numpy as np
    import torch

    import paper_1412_0659_amd as bh
    from paper_1412_0659_amd.autograd import leapfrog, surface_density
    from workloads import ics
    w = ics.DIFF_WORKLOADS[name]
    s = ics.disk_halo_scaled(w["n"], w["seed"])
    tgt_ic = ics.perturbed(s, w["target_seed"])
    dev = torch.device("cuda:0")
    sel = torch.from_numpy(s.is_disk.astype(np.uint8)).to(dev)
    tree = bh.Tree(s.n, adjoint=True, pos_fp64=True, pair_groups=pair_groups)
    # target: the density the perturbed initial conditions reach after K steps
    with torch.no_grad():
        xt, _ = leapfrog(torch.from_numpy(tgt_ic.pos).to(dev), torch.from_numpy(tgt_ic.vel).to(dev),
                         torch.from_numpy(s.mass).to(dev), tree, w["dt"], w["steps"], w["theta"],
                         w["eps"], w["every"])
        target = surface_density(xt, torch.from_numpy(s.mass).to(dev), sel, tree, w["grid"])
    x0 = torch.from_numpy(s.pos).to(dev).requires_grad_(True)
    v0 = torch.from_numpy(s.vel).to(dev).requires_grad_(True)
    m = torch.from_numpy(s.mass).to(dev).requires_grad_(True)
    # one untimed forward + reverse sweep first (allocator, code objects)
    xK, _ = leapfrog(x0, v0, m, tree, w["dt"], w["steps"], w["theta"], w["eps"], w["every"])
    ((surface_density(xK, m, sel, tree, w["grid"]) - target) ** 2).sum().backward()
    for a in (x0, v0, m):
        a.grad = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xK, _ = leapfrog(x0, v0, m, tree, w["dt"], w["steps"], w["theta"], w["eps"], w["every"])
    loss = ((surface_density(xK, m, sel, tree, w["grid"]) - target) ** 2).sum()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    fwd, bwd = t1 - t0, t2 - t1
    log(f"[bench] adjoint: forward {fwd:.2f} s, backward {bwd:.2f} s")
    finite = all(bool(torch.isfinite(a.grad).all()) for a in (x0, v0, m))
    # the same with a snapshot after every step: no segment is recomputed
    grads = [a.grad.clone() for a in (x0, v0, m)]
    for a in (x0, v0, m):
        a.grad = None
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    xK, _ = leapfrog(x0, v0, m, tree, w["dt"], w["steps"], w["theta"], w["eps"], 1)
    loss1 = ((surface_density(xK, m, sel, tree, w["grid"]) - target) ** 2).sum()
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    loss1.backward()
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    # the FP64 atomic sums of the force VJP run in a varying order, so the two
    # sweeps agree to rounding, not bit for bit
    diff = max(float((a.grad - g).abs().max() / g.abs().max())
               for a, g in zip((x0, v0, m), grads))
    # one force VJP at the initial state, its adjoint walk kernel timed by the
    # library's events around that launch (the counters' workload)
    vjp_ms, vjp_inter = vjp_kernel_ms(tree, s, w)
    tree.close()
    fwd1, bwd1 = t4 - t3, t5 - t4
    snap_mb = w["steps"] * s.n * tree.snapshot_bytes(1) / 1e6
    log(f"[bench] adjoint, snapshot every step: forward {fwd1:.2f} s, backward {bwd1:.2f} s, "
        f"gradients within {diff:.1e} of the every-8 sweep's")
    return {"workload": name, "n": s.n, "steps": w["steps"], "checkpoint_every": w["every"],
            "theta": w["theta"], "eps": w["eps"], "dt": w["dt"], "grid": list(w["grid"]),
            "loss": float(loss.detach()), "forward_s": fwd, "backward_s": bwd,
            "backward_over_forward": bwd / fwd,
            "ms_per_step_forward": 1e3 * fwd / w["steps"],
            "ms_per_step_backward": 1e3 * bwd / w["steps"], "grad_finite": finite,
            "walk_vjp_kernel_ms": vjp_ms, "walk_vjp_interactions": vjp_inter,
            "every_step_snapshots": {"forward_s": fwd1, "backward_s": bwd1,
                                     "backward_over_forward": bwd1 / fwd1,
                                     "snapshot_mb": snap_mb,
                                     "grad_max_rel_diff_vs_every_8": diff}}


def counter_report(counters, key, tflops_paper, paper_flops_per_walk):
    """FP32 (+ FP16) VALU flops of a walk kernel from the committed counters:
    the counted flops relative to the paper's convention on the profiled
    dispatch, applied to this run's rate; None without current counters."""
    c = (counters or {}).get(key)
    if not c or not (c.get("n_pp") or c.get("n_pc")):
        return None
    hw, ins = counter_flops(c)
    ref = paper_flops(c.get("n_pp", 0), c.get("n_pc", 0))
    tf = tflops_paper * hw / ref
    return {"kernel": key, "tflops_counted": tf, "frac_counted": tf / PEAK_FP32_TFLOPS,
            "tflops_fp32_instruction_classes": tflops_paper * ins / ref,
            "counted_over_paper_flops": hw / ref,
            "valu_instructions": c.get("SQ_INSTS_VALU"),
            "fma_f32": c.get("SQ_INSTS_VALU_FMA_F32"), "mul_f32": c.get("SQ_INSTS_VALU_MUL_F32"),
            "add_f32": c.get("SQ_INSTS_VALU_ADD_F32"), "trans_f32": c.get("SQ_INSTS_VALU_TRANS_F32"),
            "flops_fp16": c.get("SQ_INSTS_VALU_FLOPS_FP16"),
            "profiled_ms": c.get("mean_ms")}


def vjp_kernel_ms(tree, s, w, reps=3):
    """Adjoint walk kernel time of tree_force_vjp at the initial state of the
    differentiation workload (mean over reps after one warm-up call), and the
    interaction count of its lists."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    tree.set_state(torch.from_numpy(s.pos).to(dev), torch.from_numpy(s.vel).to(dev),
                   torch.from_numpy(s.mass).to(dev))
    u = torch.from_numpy(np.random.default_rng(77).normal(size=(s.n, 3)).astype(np.float32)).to(dev)
    gp = torch.zeros((s.n, 3), dtype=torch.float32, device=dev)
    gm = torch.zeros((s.n,), dtype=torch.float32, device=dev)
    tree.force(w["theta"], w["eps"])
    st = tree.stats()
    ms = []
    for k in range(reps + 1):
        tree.force_vjp(w["theta"], w["eps"], u, 1.0, gp, gm)
        t = tree.stats()["ms_walk_vjp"]
        if k:
            ms.append(t)
    return sum(ms) / len(ms), int(st["n_pp"] + st["n_pc"])


def profile_kernels(meta_path=None, log=print):
    """The dispatches the committed VALU counters describe: at the 13M
    workload one FP32 and one FP16 far-field walk after a warm-up of each;
    at the 1M differentiation workload's initial state one force VJP after a
    warm-up.  Writes their interaction counts to meta_path (JSON)."""
    import numpy as np
    import torch

    import paper_1412_0659_amd as bh
    from workloads import ics
    dev = torch.device("cuda:0")
    w = ics.WORKLOADS["disk_halo_13m"]
    snap = ics.make("disk_halo_13m")
    pos = torch.from_numpy(snap.pos).to(dev)
    mass = torch.from_numpy(snap.mass).to(dev)
    meta = {"workload": "disk_halo_13m", "theta": w["theta"], "eps": w["eps"], "kernels": {}}
    for f16, key in ((False, "k_walk<false, false>"), (True, "k_walk<false, true>")):
        t = bh.Tree(snap.n, far_fp16=f16)
        t.build(pos, mass)
        for _ in range(2):
            t.force(w["theta"], w["eps"])
            st = t.stats()
        log(f"[bench] profile {key}: walk {st['ms_walk']:.2f} ms")
        meta["kernels"][key] = {"n_pp": st["n_pp"], "n_pc": st["n_pc"],
                                "workload": "disk_halo_13m"}
        t.close()
    del pos, mass
    wa = ics.DIFF_WORKLOADS["disk_halo_1m_adjoint"]
    s = ics.disk_halo_scaled(wa["n"], wa["seed"])
    t = bh.Tree(s.n, adjoint=True, pos_fp64=True)
    ms, inter = vjp_kernel_ms(t, s, wa, reps=1)
    log(f"[bench] profile k_walk_vjp<false>: {ms:.2f} ms")
    meta["kernels"]["k_walk_vjp<false>"] = {"interactions": inter,
                                            "workload": "disk_halo_1m_adjoint"}
    t.close()
    if meta_path:
        with open(meta_path, "w") as f:
            json.dump(meta, f, indent=1)
    return meta


def write_counters(out_path, meta_path, dbs, command):
    """The committed counter summary: per-dispatch counters of the profiled
    walk and VJP kernels (the second, warm dispatch of each), the sources'
    hashes and the profiled interaction counts."""
    # each database holds, per walk kernel, the 13M dispatches and (FP32) one
    # at the 1M adjoint state: keep the long ones
    summ = pmc_summary(dbs, min_frac=0.5)
    with open(meta_path) as f:
        meta = json.load(f)
    kernels = {}
    for name, row in summ.items():
        for key in meta["kernels"]:
            base = key.split("<")[0]
            if name.split("(")[0].endswith(key) or (name.startswith("void bh::" + base + "<")
                                                     and key in name):
                kernels[key] = dict(row, **meta["kernels"][key])
    doc = {"command": command, "walk_source_sha256_16": walk_source_hash(),
           "vjp_source_sha256_16": walk_source_hash(VJP_SOURCES),
           "note": "counters are means per dispatch over the profiled dispatches, summed over "
                   "the chip; k_walk<·> at the 13M disk + halo workload (theta 0.4, eps 0.002), "
                   "k_walk_vjp at the 1M differentiation workload's initial state",
           "kernels": kernels}
    with open(out_path, "w") as f:
        json.dump(doc, f, indent=1)
    return doc


def counters_text(json_path):
    """The committed counter JSON as a text table: per kernel, the counters
    per dispatch, the counted flops (FLOPS counters x 64 lanes) per
    interaction and against the paper's convention, the rate at the profiled
    time and the VALU issue rate per SIMD."""
    with open(json_path) as f:
        d = json.load(f)
    lines = ["# rocprofv3 --pmc VALU instruction mix and flop counters of the walk kernels (13M disk "
             "+ halo,",
             "# theta 0.4, eps 0.002: FP32 walk and FP16 far-field walk) and of the force VJP (1M "
             "differentiation",
             "# workload's initial state); means per dispatch over the profiled dispatches, summed "
             "over the chip.",
             f"# walk source sha256/16 {d['walk_source_sha256_16']}, VJP source sha256/16 "
             f"{d['vjp_source_sha256_16']}",
             f"# command: {d['command']}; python3 bench.py --counters-text "
             f"profiles/{os.path.basename(json_path)}",
             "#   (from the repository root; OUT: any output directory; the JSON beside this file "
             "holds the same numbers)", "#"]
    simds = 256 * 4
    for name, c in d["kernels"].items():
        lines.append(f"{name}:")
        for k in sorted(k for k in c if k.startswith("SQ_")) + ["mean_ms"]:
            lines.append(f"   {k:34s} {c[k]:.4e}")
        hw, _ = counter_flops(c)
        if "interactions" in c:
            inter, paper = c["interactions"], None
        else:
            inter, paper = c["n_pp"] + c["n_pc"], paper_flops(c["n_pp"], c["n_pc"])
        tf = hw / (c["mean_ms"] * 1e-3) / 1e12
        extra = f"; / paper convention {hw / paper:.3f}" if paper else ""
        lines.append(f"   counted flops (FLOPS counters x 64) {hw:.4e}; per interaction "
                     f"{hw / inter:.1f}{extra}; at the profiled time {tf:.1f} TFLOP/s = "
                     f"{tf / PEAK_FP32_TFLOPS:.3f} of {PEAK_FP32_TFLOPS}")
        rate = c["SQ_INSTS_VALU"] / (c["mean_ms"] * 1e-3 * 2.4e9 * simds)
        lines.append(f"   VALU wave-instructions per SIMD per cycle (2.4 GHz, {simds} SIMDs) "
                     f"{rate:.3f}")
    return "\n".join(lines) + "\n"


def trace_summary(paths, top=30):
    """Per-kernel calls, mean and total duration from rocprofv3 --kernel-trace
    databases (sqlite), by total time: a text table."""
    import sqlite3
    from collections import defaultdict
    tot = defaultdict(float)
    cnt = defaultdict(int)
    for db in paths:
        con = sqlite3.connect(db)
        q = ("select ks.display_name, kd.end - kd.start from rocpd_kernel_dispatch kd "
             "join rocpd_info_kernel_symbol ks on kd.kernel_id = ks.id")
        for name, d in con.execute(q):
            short = name.replace("void ", "").split("(")[0].replace("bh::", "")
            tot[short] += d
            cnt[short] += 1
        con.close()
    grand = sum(tot.values())
    lines = [f"{'kernel':44s} {'calls':>6s} {'avg_us':>11s} {'total_ms':>10s} {'pct':>6s}"]
    for k in sorted(tot, key=lambda k: -tot[k])[:top]:
        lines.append(f"{k[:44]:44s} {cnt[k]:6d} {tot[k] / cnt[k] / 1e3:11.1f} "
                     f"{tot[k] / 1e6:10.2f} {100 * tot[k] / grand:6.2f}")
    return "\n".join(lines)


def write_traffic(out_path, fetch_db, write_db, copy_fetch_db, copy_write_db, command):
    """The committed HBM traffic of the FP32 walk: FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch, mean over the walk's dispatches) scaled by what the
    same counters read for the plain 1 GiB device copy of --copy-calibration."""
    key = "k_walk<false, false>"

    def mean_of(db, counter, pat):
        rows = [r for n, r in pmc_summary([db]).items() if pat in n]
        vals = [r[counter] for r in rows if counter in r]
        disp = sum(r["dispatches"] for r in rows)
        return (sum(v * r["dispatches"] for v, r in zip(vals, rows)) / disp if disp else None,
                disp)

    f, nf = mean_of(fetch_db, "FETCH_SIZE", "k_walk<false, false>")
    w_, nw = mean_of(write_db, "WRITE_SIZE", "k_walk<false, false>")
    cf, _ = mean_of(copy_fetch_db, "FETCH_SIZE", "copyBuffer")
    cw, _ = mean_of(copy_write_db, "WRITE_SIZE", "copyBuffer")
    gib = float(1 << 30)
    ff, wf = gib / (cf * 1024.0), gib / (cw * 1024.0)
    doc = {"kernel": key, "workload": "disk_halo_13m", "walk_source_sha256_16": walk_source_hash(),
           "fetch_size_kib_per_dispatch": f, "write_size_kib_per_dispatch": w_,
           "dispatches": [nf, nw],
           "copy_calibration": {"bytes_read": gib, "bytes_written": gib, "fetch_size_kib": cf,
                                "write_size_kib": cw, "fetch_factor": ff, "write_factor": wf},
           "hbm_bytes_per_launch": f * 1024.0 * ff + w_ * 1024.0 * wf,
           "hbm_fetch_bytes_per_launch": f * 1024.0 * ff,
           "hbm_write_bytes_per_launch": w_ * 1024.0 * wf, "command": command}
    with open(out_path, "w") as fh:
        json.dump(doc, fh, indent=1)
    return doc


def domains(name="disk_halo_13m", ps=(2, 4, 8, 16), curve="ph", max_boundary=4096, reps=3,
            log=print, sampling=None, snap=None):
    """The force evaluation split into p spatial domains on the one device
    (Sec. III.B): flop-weighted cuts, per-domain trees in the global box,
    boundary trees, merged local essential trees, own + LET walks; against
    one tree over all particles."""
    import numpy as np
    import torch

    import paper_1412_0659_amd as bh
    from workloads import ics
    w = ics.WORKLOADS[name]
    theta, eps = w["theta"], w["eps"]
    if snap is None:
        snap = ics.make(name)
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(snap.pos).to(dev)
    mass = torch.from_numpy(snap.mass).to(dev)
    one = bh.Tree(snap.n, curve=curve)
    one.build(pos, mass)
    ms1, acc1, _, st1 = _timed_force(one, theta, eps, reps)
    inter1 = st1["n_pp"] + st1["n_pc"]
    a1 = torch.empty((snap.n, 3), dtype=torch.float32, device=dev)
    p1 = torch.empty((snap.n,), dtype=torch.float32, device=dev)
    calls = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        one.force(theta, eps, a1, p1)
        e1.record()
        torch.cuda.synchronize()
        calls.append(e0.elapsed_time(e1))
    call1 = float(np.median(calls))
    one.close()
    sample = np.arange(0, snap.n, 211)
    ref = acc1[sample]
    rows = []
    for p in ps:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        smp = None
        if sampling:
            px = max(v for v in range(1, int(p ** 0.5) + 1) if p % v == 0)
            smp = (px, p // px, sampling, sampling)
        d = bh.Domains(pos, mass, p, theta, eps, max_boundary=max_boundary, curve=curve,
                       sampling=smp)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        info = d.build_lets()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        acc, pot = d.forces()
        times, per_dom, conc = [], [], []
        for _ in range(reps):
            # one stream, domain after domain: per-domain times
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(d.trees) + 1)]
            ev[0].record()
            for k, (t, ids) in enumerate(zip(d.trees, d.ids)):
                t.force_let(theta, eps, rows=ids, acc=acc, pot=pot)
                ev[k + 1].record()
            torch.cuda.synchronize()
            times.append(ev[0].elapsed_time(ev[-1]))
            per_dom.append([ev[k].elapsed_time(ev[k + 1]) for k in range(len(d.trees))])
            # the domains on four streams at once
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            d.forces(acc=acc, pot=pot)
            e1.record()
            torch.cuda.synchronize()
            conc.append(e0.elapsed_time(e1))
        ms_serial = float(np.median(times))
        ms = float(np.median(conc))
        dom_ms = np.median(np.asarray(per_dom), axis=0)
        inter = 0
        for t in d.trees:
            st = t.stats()
            inter += st["n_pp"] + st["n_pc"]
        err = _rel(acc.double().cpu().numpy()[sample], ref)
        allinfo = np.concatenate([i for i in info if len(i)]) if p > 1 else np.zeros((0, 3))
        let_cells = int(allinfo[:, 1].sum()) if len(allinfo) else 0
        let_parts = int(allinfo[:, 2].sum()) if len(allinfo) else 0
        row = {"p": p, "cut": "exact" if smp is None else
               f"sampled {smp[0]}x{smp[1]}, {smp[2]} samples per process and level",
               "cuts_sizes": np.diff(d.cuts).tolist(), "setup_s": t1 - t0,
               "let_build_s": t2 - t1, "force_ms": ms, "force_ms_one_stream": ms_serial,
               "domain_ms_max": float(dom_ms.max()),
               "domain_ms_min": float(dom_ms.min()),
               "interactions": int(inter), "interactions_over_one_tree": inter / inter1,
               "interactions_per_s": inter / (ms * 1e-3),
               "tflops": paper_flops(sum(t.stats()["n_pp"] for t in d.trees),
                                     sum(t.stats()["n_pc"] for t in d.trees)) / (ms * 1e-3) / 1e12,
               "boundary_sufficed": int(allinfo[:, 0].sum()) if len(allinfo) else 0,
               "pairs": p * (p - 1), "let_cells": let_cells, "let_particles": let_parts,
               "acc_rel_diff_vs_one_tree_median": float(np.median(err)),
               "acc_rel_diff_vs_one_tree_p99": float(np.percentile(err, 99))}
        log(f"[bench] domains p={p} ({row['cut']}): force {ms:.1f} ms on 4 streams, "
            f"{ms_serial:.1f} ms on one (one tree {call1:.1f}), slowest/fastest domain "
            f"{dom_ms.max():.2f}/{dom_ms.min():.2f} ms, "
            f"interactions x{inter / inter1:.3f}, LET build {t2 - t1:.3f} s "
            f"({let_cells} cells, {let_parts} particles), "
            f"boundary trees {row['boundary_sufficed']}/{row['pairs']}")
        rows.append(row)
        d.close()
    return {"workload": name, "n": snap.n, "theta": theta, "eps": eps, "curve": curve,
            "max_boundary": max_boundary, "one_tree_walk_ms": ms1, "one_tree_force_ms": call1,
            "one_tree_interactions": int(inter1), "rows": rows}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="disk_halo_13m")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--curve", choices=("morton", "ph"), default="morton",
                    help="space-filling curve of the keys (the same cells either way)")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-domains", action="store_true")
    ap.add_argument("--precision-sweep", action="store_true",
                    help="only run the precision form's table (4M disk + halo, theta 0.3/0.4/0.6)")
    ap.add_argument("--param-sweep", action="store_true",
                    help="only run the walk cost sweep over theta and (nleaf, ncrit) at 4M")
    ap.add_argument("--domains", type=str, default=None,
                    help="comma-separated domain counts: time the multi-domain force "
                         "(own + local-essential-tree walks) instead")
    ap.add_argument("--max-boundary", type=int, default=4096,
                    help="with --domains: cell budget of each boundary tree")
    ap.add_argument("--sampling", type=int, default=0,
                    help="with --domains: cut by the two-level sampling with this many "
                         "samples per process and level (0: exact cut)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only run the differentiation workload and print its JSON object")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy five times (the "
                         "reference kernel for scaling the HBM byte counters)")
    ap.add_argument("--no-c4", action="store_true",
                    help="skip the 4M precision sweep over theta 0.3 / 0.4 / 0.6")
    ap.add_argument("--pair-groups", type=int, default=0,
                    help="time the steps with paired target sets (bh_params.pair_groups; "
                         "0 = the groups of the method, the default)")
    ap.add_argument("--no-pairs", action="store_true",
                    help="skip the paired-target-set runs (walks at pair_groups 32, 48, 64; "
                         "the adjoint at 48)")
    ap.add_argument("--no-param-sweep", action="store_true",
                    help="skip the walk cost curve over theta, nleaf and ncrit")
    ap.add_argument("--profile-kernels", type=str, default=None, metavar="META_JSON",
                    help="only run the dispatches the committed VALU counters describe "
                         "(run under rocprofv3 --pmc); write their interaction counts here")
    ap.add_argument("--pmc-summary", nargs="+", default=None, metavar="DB",
                    help="only print the per-kernel mean counters of rocprofv3 databases "
                         "(dispatches at least half as long as the kernel's longest)")
    ap.add_argument("--write-counters", nargs="+", default=None, metavar="ARG",
                    help="OUT_JSON META_JSON DB...: write the committed counter summary")
    ap.add_argument("--trace-summary", nargs="+", default=None, metavar="DB",
                    help="only print the per-kernel time table of rocprofv3 --kernel-trace "
                         "databases")
    ap.add_argument("--write-traffic", nargs=5, default=None, metavar="ARG",
                    help="OUT_JSON FETCH_DB WRITE_DB COPY_FETCH_DB COPY_WRITE_DB: write the "
                         "committed walk traffic summary")
    ap.add_argument("--counters-text", nargs=2, default=None, metavar=("JSON", "OUT"),
                    help="render the committed counter JSON as the text table")
    ap.add_argument("--write-build-traffic", nargs=4, default=None,
                    metavar=("OUT", "FETCH_DB", "WRITE_DB", "BENCH_JSON"),
                    help="write the build-phase HBM bytes summary from two --pmc runs")
    ap.add_argument("--quiet", action="store_true")
    args = ap.parse_args(argv)
    if args.trace_summary:
        print(trace_summary(args.trace_summary))
        return 0
    if args.pmc_summary:
        print(json.dumps(pmc_summary(args.pmc_summary, min_frac=0.5), indent=1))
        return 0
    if args.write_traffic:
        out, dbs = args.write_traffic[0], args.write_traffic[1:]
        print(json.dumps(write_traffic(out, *dbs, os.environ.get("BH_PROFILE_COMMAND", "")),
                         indent=1))
        return 0
    if args.counters_text:
        text = counters_text(args.counters_text[0])
        with open(args.counters_text[1], "w") as f:
            f.write(text)
        print(text)
        return 0
    if args.write_build_traffic:
        out, f_db, w_db, bj = args.write_build_traffic
        print(write_build_traffic(out, f_db, w_db, bj, os.environ.get("BH_PROFILE_COMMAND", "")))
        return 0
    if args.write_counters:
        out, meta, dbs = args.write_counters[0], args.write_counters[1], args.write_counters[2:]
        cmd = os.environ.get("BH_PROFILE_COMMAND", "")
        print(json.dumps(write_counters(out, meta, dbs, cmd), indent=1))
        return 0

    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the "
              "library runs on one GPU (several spatial domains run as contexts on that "
              "device, --domains; the exchange between GPUs is not implemented)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1412_0659_amd as bh
    from workloads import ics

    if args.copy_calibration:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4,
                          "launches": 5}))
        return 0

    log = (lambda *a: None) if args.quiet else (lambda *a: print(*a, file=sys.stderr, flush=True))
    if args.profile_kernels:
        profile_kernels(args.profile_kernels, log=log)
        return 0
    if args.adjoint_only:
        print(json.dumps(adjoint(log=log)))
        return 0
    if args.precision_sweep:
        r = precision_sweep(log=log)
        r.pop("_anchor")
        print(json.dumps(r))
        return 0
    if args.param_sweep:
        print(json.dumps(param_sweep(log=log)))
        return 0
    if args.domains:
        ps = tuple(int(v) for v in args.domains.split(","))
        print(json.dumps(domains(args.workload, ps, args.curve, args.max_boundary, log=log,
                                 sampling=args.sampling or None)))
        return 0

    w = ics.WORKLOADS[args.workload]
    theta, eps, dt = w["theta"], w["eps"], w.get("dt", 1e-3)
    t0 = time.perf_counter()
    snap = ics.make(args.workload)
    log(f"[bench] workload {args.workload} n={snap.n} generated in {time.perf_counter() - t0:.1f} s")

    dev = torch.device("cuda:0")
    pos = torch.from_numpy(snap.pos).to(dev)
    vel = torch.from_numpy(snap.vel).to(dev)
    mass = torch.from_numpy(snap.mass).to(dev)
    tree = bh.Tree(snap.n, curve=args.curve, pair_groups=args.pair_groups)
    tree.set_state(pos, vel, mass)
    tree.sync()
    for k in range(args.warmup):
        tree.step(dt, theta, eps)
        tree.sync()
        log(f"[bench] warmup step {k} done")

    torch.cuda.synchronize()
    per = []
    t_start = time.perf_counter()
    for k in range(args.steps):
        tree.step(dt, theta, eps)
        per.append(tree.stats())       # synchronises the stream
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    log(f"[bench] {args.steps} timed steps in {wall:.3f} s")

    n_pp = sum(s["n_pp"] for s in per)
    n_pc = sum(s["n_pc"] for s in per)
    walk_ms = sum(s["ms_walk"] for s in per)
    inter = n_pp + n_pc
    flops = paper_flops(n_pp, n_pc)
    walk_tflops = flops / (walk_ms * 1e-3) / 1e12
    last = per[-1]
    out = {
        "metric": "tree-walk interactions/s & Tflops at N=13M, θ=0.4; FP16-far vs FP32 at force err",
        "value": inter / wall,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": snap.n, "theta": theta, "eps": eps, "dt": dt,
                   "nleaf": 16, "ncrit": 64, "curve": args.curve, "pair_groups": args.pair_groups,
                   "model": "exponential disk + Hernquist halo"
                   if w["model"] == "disk_halo" else "Plummer sphere"},
        "tflops_step": flops / wall / 1e12,
        "tflops_walk": walk_tflops,
        "interactions_per_s_walk": inter / (walk_ms * 1e-3),
        "pp_per_particle": n_pp / args.steps / snap.n,
        "pc_per_particle": n_pc / args.steps / snap.n,
        "ms_phase": {"sort": np.mean([s["ms_sort"] for s in per]),
                     "build": np.mean([s["ms_build"] for s in per]),
                     "moments": np.mean([s["ms_moments"] for s in per]),
                     "walk": walk_ms / args.steps,
                     "step_events": np.mean([s["ms_step"] for s in per])},
        "tree": {"cells": last["ncells"], "leaves": last["nleaves"], "groups": last["ngroups"],
                 "depth": last["depth"]},
        "hbm_phases": hbm_phases(snap.n, last["ncells"],
                                 float(np.mean([s["ms_sort"] for s in per])),
                                 float(np.mean([s["ms_moments"] for s in per])),
                                 ms_build=float(np.mean([s["ms_build"] for s in per])),
                                 depth=last["depth"]),
        "paper_context": {"hardware": "NVIDIA K20X, the paper's 1-GPU column (Table II)",
                          "workload": "the paper's Milky Way model, 13M particles, theta 0.4",
                          "gravity_interactions_per_s": 3.33e10, "gravity_tflops": 1.77,
                          "note": "another machine and another model: context, not a baseline"},
        "roofline": {"bound": "alu", "achieved": walk_tflops, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": walk_tflops / PEAK_FP32_TFLOPS,
                     # the committed counters profile the walk over the method's groups
                     "traffic": None if args.pair_groups else load_traffic(), "kernel": "k_walk",
                     "flops_convention": "23 per p-p, 65 per p-c (paper Sec. VI.A)"},
    }
    tree.close()
    del pos, vel, mass
    counters = load_counters()
    out["valu_counters"] = None if args.pair_groups else counter_report(
        counters, "k_walk<false, false>", walk_tflops, paper_flops(n_pp, n_pc) / args.steps)
    anchors = []
    if not args.no_precision:
        out["precision"] = precision(snap, theta, eps, log=log)
        ref = out["precision"].pop("_ref")
        a = out["precision"].pop("_anchor")
        if not args.no_pairs:
            out["paired_target_sets"] = paired_sets(snap, theta, eps, ref, a["idx"],
                                                    out["precision"]["fp32"]["walk_ms"], log=log)
        a["name"] = f"{args.workload} theta {theta}"
        anchors.append(a)
        f16 = out["precision"]["fp16_far"]
        f16["valu_counters"] = counter_report(counters, "k_walk<false, true>", f16["tflops_walk"],
                                              paper_flops(f16["n_pp"], f16["n_pc"]))
    if not args.no_c4:
        c4 = precision_sweep(log=log)
        a = c4.pop("_anchor")
        if a is not None:
            a["name"] = f"{c4['workload']} theta 0.4"
            anchors.append(a)
        out["precision_c4"] = c4
    if not args.no_param_sweep:
        out["param_sweep"] = param_sweep(log=log)
    if not args.no_adjoint:
        out["adjoint"] = adjoint(log=log)
        ad = out["adjoint"]
        if not args.no_pairs:
            p48 = adjoint(log=log, pair_groups=48)
            ad["paired_target_sets_48"] = {
                k: p48[k] for k in ("forward_s", "backward_s", "backward_over_forward",
                                    "walk_vjp_kernel_ms", "walk_vjp_interactions")}
            ad["paired_target_sets_48"]["every_step_backward_over_forward"] = \
                p48["every_step_snapshots"]["backward_over_forward"]
        c = (counters or {}).get("k_walk_vjp<false>")
        rep = None
        if c and c.get("interactions"):
            hw, ins = counter_flops(c)
            # the counted flops per interaction of the profiled dispatch, applied
            # to this run's lists and kernel time
            per = hw / c["interactions"]
            tf = per * ad["walk_vjp_interactions"] / (ad["walk_vjp_kernel_ms"] * 1e-3) / 1e12
            rep = {"kernel": "k_walk_vjp", "bound": "alu", "achieved": tf,
                   "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": tf / PEAK_FP32_TFLOPS,
                   "counter_flops_per_interaction": per,
                   "instruction_flops_per_interaction": ins / c["interactions"],
                   "convention": "hardware FP32 VALU flop counters (SQ_INSTS_VALU_FLOPS_FP32 "
                                 "+ _TRANS, x 64 lanes) of the profiled dispatch per interaction"}
        ad["roofline_walk_vjp"] = rep
    if not args.no_domains:
        r = domains(args.workload, (8,), args.curve, log=log, snap=snap)
        row = r["rows"][0]
        out["domains"] = {
            "what": "the same force split into 8 spatial domains on this GPU: flop-weighted "
                    "cuts, per-domain trees in the global box, boundary trees, merged local "
                    "essential trees; own + LET walks of the domains on 4 streams",
            "p": 8, "force_ms": row["force_ms"], "one_tree_force_ms": r["one_tree_force_ms"],
            "force_ms_one_stream": row["force_ms_one_stream"],
            "domain_ms_max": row["domain_ms_max"], "domain_ms_min": row["domain_ms_min"],
            "interactions_over_one_tree": row["interactions_over_one_tree"],
            "let_build_s": row["let_build_s"], "let_cells": row["let_cells"],
            "let_particles": row["let_particles"],
            "boundary_sufficed": row["boundary_sufficed"], "pairs": row["pairs"],
            "acc_rel_diff_vs_one_tree_median": row["acc_rel_diff_vs_one_tree_median"]}
    if not args.no_cpu_baseline:
        log("[bench] CPU baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(snap, theta, eps)
        if anchors:
            log("[bench] oracle anchors of the force errors ...")
            out["cpu_baseline"]["oracle_anchors"] = oracle_anchors(anchors)
        log("[bench] oracle on the other workloads ...")
        out["cpu_baseline"]["configs"] = cpu_configs(anchors)
    out["ms_phase"] = {k: float(v) for k, v in out["ms_phase"].items()}
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
