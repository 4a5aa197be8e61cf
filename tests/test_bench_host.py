"""Host logic of bench.py: the rocprofv3 database readers and the byte and
flop bookkeeping behind the bench line (no GPU)."""
import json
import os
import sqlite3

import bench


def _db(path, dispatches):
    """A database with the subset of the rocprofv3 (rocpd) schema the readers
    use; dispatches: [(kernel, {counter: value}), ...] in launch order."""
    con = sqlite3.connect(path)
    con.executescript(
        "create table rocpd_info_kernel_symbol (id integer primary key, display_name text);"
        "create table rocpd_info_pmc (id integer primary key, name text);"
        "create table rocpd_kernel_dispatch (id integer primary key, event_id integer, "
        "kernel_id integer, start integer, end integer);"
        "create table rocpd_pmc_event (id integer primary key, event_id integer, pmc_id integer, "
        "value real);")
    syms, pmcs = {}, {}
    for did, (kernel, counters) in enumerate(dispatches):
        kid = syms.setdefault(kernel, len(syms) + 1)
        con.execute("insert or ignore into rocpd_info_kernel_symbol values (?, ?)", (kid, kernel))
        con.execute("insert into rocpd_kernel_dispatch values (?, ?, ?, ?, ?)",
                    (did + 1, 100 + did, kid, 1000 * did, 1000 * did + 500))
        for name, val in counters.items():
            pid = pmcs.setdefault(name, len(pmcs) + 1)
            con.execute("insert or ignore into rocpd_info_pmc values (?, ?)", (pid, name))
            # two rows per dispatch (per-XCD partial values) that the reader sums
            con.execute("insert into rocpd_pmc_event (event_id, pmc_id, value) values (?, ?, ?)",
                        (100 + did, pid, val / 2))
            con.execute("insert into rocpd_pmc_event (event_id, pmc_id, value) values (?, ?, ?)",
                        (100 + did, pid, val / 2))
    con.commit()
    con.close()


def _build(scale):
    c = lambda v: {"FETCH_SIZE": v * scale}  # noqa: E731
    return [("void bh::k_bbox_partial(float const*)", c(1)), ("void bh::k_keys<false>(x)", c(2)),
            ("void bh::k_sort_count(x)", c(3)), ("void bh::k_scan_reduce(x)", c(4)),
            ("void bh::k_sort_scatter(x)", c(5)), ("void bh::k_gather(x)", c(6)),
            ("void bh::k_lb_table(x)", c(7)), ("void bh::k_scan_reduce(x)", c(8)),
            ("void bh::k_group_fill(x)", c(9)), ("void bh::k_moments_level(x)", c(10)),
            ("void bh::k_moments_tail(x)", c(11)), ("void bh::k_moments_level(x)", c(12))]


def test_build_phase_counters_split_one_build(tmp_path):
    db = str(tmp_path / "run_results.db")
    rows = _build(1) + [("void bh::k_walk<false, false>(x)", {"FETCH_SIZE": 1000})] + _build(100) \
        + [("void bh::k_walk_prep(x)", {"FETCH_SIZE": 5})]
    _db(db, rows)
    got = bench.pmc_rows(db)
    assert [r["kernel"] for r in got] == [k for k, _ in rows]
    assert got[1]["FETCH_SIZE"] == 2 and abs(got[0]["ms"] - 5e-4) < 1e-12
    out, kernels = bench.build_phase_counters(db, "FETCH_SIZE", build_index=1)
    # sort: bbox .. gather; build: up to the first moments kernel; moments: the rest
    assert out == {"sort": 100 * (1 + 2 + 3 + 4 + 5 + 6), "build": 100 * (7 + 8 + 9),
                   "moments": 100 * (10 + 11 + 12)}
    assert kernels["build"] == ["k_lb_table", "k_scan_reduce", "k_group_fill"]
    assert bench.build_phase_counters(db, "FETCH_SIZE", 0)[0]["moments"] == 33
    per_kernel = bench.pmc_summary([db])
    assert per_kernel["void bh::k_walk<false, false>(x)"]["FETCH_SIZE"] == 1000


def test_counter_flops_count_per_lane():
    c = {"SQ_INSTS_VALU_FLOPS_FP32": 10.0, "SQ_INSTS_VALU_FLOPS_FP32_TRANS": 1.0,
         "SQ_INSTS_VALU_FMA_F32": 3.0, "SQ_INSTS_VALU_MUL_F32": 2.0, "SQ_INSTS_VALU_ADD_F32": 1.0,
         "SQ_INSTS_VALU_TRANS_F32": 1.0}
    hw, ins = bench.counter_flops(c)
    assert hw == 64 * 11 and ins == 64 * (2 * 3 + 2 + 1 + 1)


def test_phase_bytes():
    p = bench.hbm_phases(1000, 300, 2.0, 1.0, ms_build=0.5, depth=10)
    assert p["sort"]["bytes"] == 1000 * 376
    assert p["moments"]["bytes"] == 1000 * 16 + 300 * 260
    assert p["build"]["bytes"] == 1000 * 8 * 10 + 300 * 40 + 1000 * 12
    assert abs(p["moments"]["GBps"] - p["moments"]["bytes"] / 1e-3 / 1e9) < 1e-9


def test_committed_counters_render(tmp_path):
    path = os.path.join(bench.ROOT, "profiles", "walk_valu_counters_disk_halo_13m.json")
    with open(path) as f:
        d = json.load(f)
    text = bench.counters_text(path)
    assert d["command"] in text
    for name in d["kernels"]:
        assert f"{name}:" in text
