"""Host logic of the measurement tools, on the CPU: the rocprofv3 summaries
(profsum) on small synthetic result databases with the profiler's schema, and
the byte models bench.py prices kernels with, against the sizes they must
reproduce (the workload's limbs and digits; the committed counter tables
confirm them within 1 %)."""
import sqlite3

import pytest

import bench
from paper_2503_22227_amd import profsum


def _db(path, kernels, events):
    con = sqlite3.connect(path)
    con.execute("create table kernels (dispatch_id integer, name text, duration integer, vgpr_count integer, "
                "accum_vgpr_count integer, lds_size integer, scratch_size integer, grid_x integer, "
                "grid_y integer, grid_z integer)")
    con.execute("create table pmc_events (name text, dispatch_id integer, counter_name text, counter_value real)")
    con.executemany("insert into kernels values (?,?,?,?,?,?,?,?,?,?)", kernels)
    con.executemany("insert into pmc_events values (?,?,?,?)", events)
    con.commit()
    con.close()
    return str(path)


def test_valu_summary(tmp_path):
    # two dispatches of 1 us (2400 cycles at 2.4 GHz), 2048 threads, each counter
    # reported by two instances: 307200 VALU wave-instructions x 4 cycles fill half
    # of 1024 SIMDs x 2400 cycles; 1228800 quad-cycles of waves = 2 waves per SIMD
    kernels = [(d, "void rf::k_a(unsigned long*)", 1000, 64, 0, 34816, 0, 2048, 1, 1) for d in (1, 2)]
    events = []
    for d in (1, 2):
        for c, v in (("SQ_INSTS_VALU", 153600.0), ("SQ_WAVE_CYCLES", 614400.0), ("SQ_INSTS_LDS", 1000.0)):
            events += [("k_a", d, c, v), ("k_a", d, c, v)]
    db = _db(tmp_path / "v.db", kernels, events)
    rows = [l for l in profsum.valu(db).splitlines() if l.startswith("| k_a")]
    assert rows == ["| k_a | 2 | 1.00 | 34816 | 0 | 32 | 0.31 | 0.50 | 2.00 | 2000 |"]


def test_traffic_scaling(tmp_path):
    # the copy of 256 MiB reads FETCH_SIZE = 128 MiB and WRITE_SIZE = 256 MiB: scales 2 and 1
    copy = [(1, "__amd_rocclr_copyBuffer", 1, 0, 0, 0, 0, 1, 1, 1)]
    cf = _db(tmp_path / "cf.db", copy, [("__amd_rocclr_copyBuffer", 1, "FETCH_SIZE", 131072.0)])
    cw = _db(tmp_path / "cw.db", copy, [("__amd_rocclr_copyBuffer", 1, "WRITE_SIZE", 262144.0)])
    k = [(1, "k_a", 1, 0, 0, 0, 0, 1, 1, 1), (2, "k_a", 1, 0, 0, 0, 0, 1, 1, 1)]
    f = _db(tmp_path / "f.db", k, [("k_a", 1, "FETCH_SIZE", 100.0), ("k_a", 2, "FETCH_SIZE", 100.0)])
    w = _db(tmp_path / "w.db", k, [("k_a", 1, "WRITE_SIZE", 50.0), ("k_a", 2, "WRITE_SIZE", 50.0)])
    text = profsum.traffic(f, w, cf, cw, 256 << 20)
    assert "scale 2.0000" in text and "scale 1.0000" in text
    assert "| k_a | 2 | 100.0 | 50.0 | 0.20 | 0.05 | 0.26 |" in text.splitlines()


N16 = 1 << 16
LIMB = 8 * N16


def test_inner_product_bytes():
    # 24 Q-limbs, 4 special, alpha = 8: 3 digits; per limb of Q u P 2 ModUp sources
    # (own digit: a, b or the gathered ciphertext instead) + 6 key limbs + 2 outputs
    hm = bench.algorithmic_bytes("inner_product", 24, 4, 8, N16, "hmult")
    ro = bench.algorithmic_bytes("inner_product", 24, 4, 8, N16, "rotate")
    assert hm == (24 * (2 + 4 + 6 + 2) + 4 * (3 + 6 + 2)) * LIMB
    assert ro == (24 * (2 + 2 + 6 + 2) + 4 * (3 + 6 + 2)) * LIMB
    assert (hm + ro) / 2 == pytest.approx(186.6e6, rel=1e-3)


def test_modup_and_pass_bytes():
    # ModUp: 24 limbs read, 3 digits x (16 + 4) extended limbs written
    assert bench.algorithmic_bytes("modup_bconv", 24, 4, 8, N16, "hmult") == (24 + 60) * LIMB
    # ModDown row pass with its tail: 48 limbs; conv and the folded ip read, out written; 24 tables
    limbs, by = bench._ntt_launch_model("ntt_fwd_rows_moddown", 24, 4, 8, N16)
    assert limbs == 48 and by == 6 * 24 * LIMB + 24 * 16 * N16
    # ModUp column pass: 60 limbs read and written once
    limbs, by = bench._ntt_launch_model("ntt_fwd_cols", 24, 4, 8, N16)
    assert limbs == 60 and by == 2 * 60 * LIMB


def test_bench_refuses_more_than_one_gpu():
    # the multi-GPU layout is described, not built: the bench says so and exits 2
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    res = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                         stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=120)
    assert res.returncode == 2
    assert "single MI355X" in res.stdout and "--gpus 2" in res.stdout


def test_batch_stage_bytes_one_item():
    """One item at N = 2^12, 9 limbs, K = 4, alpha = 8 (digits of 8 and 1 limbs):
    the ModUp extension has (9 - 8 + 4) + (9 - 1 + 4) = 17 limbs; every stage's
    bytes follow from the limb counts and one twiddle table per distinct prime."""
    n = 1 << 12
    limb, tw = 8.0 * n, 16.0 * n
    b = bench.batch_stage_bytes([(12, 9)], q_count=24, K=4, alpha=8)
    assert b["batch_ntt_fwd_cols"] == 2 * 17 * limb
    assert b["batch_ntt_fwd_rows"] == 2 * 17 * limb + tw * (9 + 4)
    assert b["batch_ntt_inv_rows_tensor"] == 3 * 9 * limb + tw * 9
    assert b["batch_ntt_inv_cols"] == 2 * 9 * limb + 2 * 8 * limb
    assert b["batch_ntt_inv_rows"] == 2 * 8 * limb + tw * 4
    assert b["batch_ntt_fwd_cols_moddown"] == (8 + 18) * limb
    assert b["batch_ntt_fwd_rows_moddown"] == 6 * 9 * limb + tw * 9
    assert b["batch_inner_product"] == bench.algorithmic_bytes("inner_product", 9, 4, 8, n, "hmult")
    assert b["batch_modup_bconv"] == bench.algorithmic_bytes("modup_bconv", 9, 4, 8, n, "hmult") == (9 + 17) * limb


def test_batch_stage_bytes_share_tables_per_degree():
    # two items of one degree share each prime's row table; a third degree adds its own
    one = bench.batch_stage_bytes([(13, 8)], 24, 4, 8)
    two = bench.batch_stage_bytes([(13, 8), (13, 8)], 24, 4, 8)
    tw13 = 16.0 * (1 << 13)
    assert two["batch_ntt_fwd_rows"] == 2 * one["batch_ntt_fwd_rows"] - tw13 * (8 + 4)
    mixed = bench.batch_stage_bytes([(13, 8), (14, 8)], 24, 4, 8)
    assert mixed["batch_ntt_inv_rows"] == one["batch_ntt_inv_rows"] + 2 * one["batch_ntt_inv_rows"]


def test_micro_summary(tmp_path):
    line = ('{"ntt_microbench": "x", "limbs": {"56": {"ntt_fwd_cols": {"avg_us": 22.0, "us_per_limb": 0.3929, '
            '"valu_frac_24ops": 0.4, "mb": 58.7, "hbm_frac": 0.3335}}, "28": {"ntt_fwd_cols": {"avg_us": 14.0, '
            '"us_per_limb": 0.5, "valu_frac_24ops": 0.3, "mb": 29.4, "hbm_frac": 0.2625}}}}')
    p = tmp_path / "m.json"
    p.write_text("noise\n" + line + "\n")
    rows = [l for l in profsum.micro(str(p)).splitlines() if l.startswith("| ntt")]
    assert rows == ["| ntt_fwd_cols | 28 | 14.00 | 0.5000 | 29.4 | 0.263 | 0.300 |",
                    "| ntt_fwd_cols | 56 | 22.00 | 0.3929 | 58.7 | 0.334 | 0.400 |"]
