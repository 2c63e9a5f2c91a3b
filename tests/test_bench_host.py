"""Host-side checks of the benchmark script: the one-GPU contract and the
figures it quotes from the paper's tables (no GPU needed)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr and r.stdout.strip() == ""


def test_paper_tables_quoted_by_the_benchmark():
    """The paper's numbers carried as context: iterations of Table thick_ring and
    Table quarterofring, and the FD direct-solver seconds of Table cube, against
    the golden copies of those tables."""
    sys.path.insert(0, ROOT)
    import bench
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_tables.json")))
    for key, (it, sec) in gold["thick_ring"].items():
        E, p = map(int, key.split(","))
        assert bench.PAPER_RING[(E, p)]["iters"] == it and bench.PAPER_RING[(E, p)]["s"] == sec
    for key, (it, sec) in gold["quarterofring"].items():
        E, p = map(int, key.split(","))
        assert bench.PAPER_ANNULUS[(E, p)] == (it, sec)
    for p, row in gold["cube_fd_s"].items():
        for E, sec in row.items():
            assert bench.PAPER_CUBE_FD_S[int(p)][int(E)] == sec


def test_committed_counter_summary_matches_the_a_product_source():
    """The benchmark's roofline.traffic comes from the committed counter
    summary of the tiled A product only while its source hash matches;
    a changed source without re-taken counters would report null."""
    sys.path.insert(0, ROOT)
    import bench
    summary = os.path.join(ROOT, "profiles", "k_spmv_tile__thick_ring_128_p3__hbm_counters.md")
    tag = [ln.split(": ", 1)[1].strip() for ln in open(summary) if ln.strip().startswith("traffic_kernel: ")][0]
    assert tag.startswith("tile ")  # tile lines and threads per block of the measured launch
    traffic, source = bench.profiled_traffic(tag, "thick_ring E=128 p=3")
    assert source is not None and source.startswith("profiles")
    # one igafd_apply_A moves more than its algorithmic bytes (x once, each stored value once)
    E, p = 128, 3
    n = E + p
    N = n ** 3
    assert traffic > 8 * N * 3 and traffic < 3 * 2.872e9
