"""Host logic of bench.py (no GPU): the one-GPU refusal and the algorithmic
flop model behind the roofline line."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2, (r.returncode, r.stderr[-500:])
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_flop_model_per_pair():
    """F_pair = N (F_A + F_B) + 2p^2 + 2pq + 40 with the nominal costs of the
    special functions (Phi 40, Phi^-1 50, scaled accumulation 20 flops):
    integral A draws q - 1 coordinates, integral B all q and adds the moment
    sums q(q+1) + 4q.  At p = q = 4, N = 4096 that is 3,219,560 flops."""
    import bench
    assert bench.NOMINAL_COSTS == {"phi": 40, "phiinv": 50, "acc": 20}
    assert bench.flops_per_pair(4, 4, 4096) == 3219560
    # by hand for p = q = 1, N = 1: A = 1+1+40+0+20, B = 1+1+40+50+2+4+20
    assert bench.flops_per_pair(1, 1, 1) == 62 + 118 + 2 + 2 + 40
    # linear in N with slope F_A + F_B
    d = bench.flops_per_pair(6, 6, 2) - bench.flops_per_pair(6, 6, 1)
    q = 6
    fa = q * q + q + 40 * q + 50 * (q - 1) + 20
    fb = q * q + q + 40 * q + 50 * q + q * (q + 1) + 4 * q + 20
    assert d == fa + fb
    # measured per-call costs enter the same formula
    c = {"phi": 30, "phiinv": 70, "acc": 3}
    assert bench.flops_per_pair(1, 1, 1, c) == (2 + 30 + 3) + (2 + 30 + 70 + 2 + 4 + 3) + 44


def test_source_digest_gates_the_counter_fields():
    """roofline.traffic and the measured cost model apply only to the kernel
    sources they were taken on: the digest covers every source the pair
    kernels and the cost probes are compiled from (every header the pair
    translation unit includes from the package)."""
    import re
    import bench
    d = bench.kernel_sources_digest()
    assert len(d) == 16 and d == bench.kernel_sources_digest()
    csrc = os.path.join(ROOT, "paper_2005_06848_amd", "csrc")
    seen, todo = set(), ["cfust_pairs.hip"]
    while todo:
        f = todo.pop()
        if f in seen:
            continue
        seen.add(f)
        with open(os.path.join(csrc, f)) as fh:
            todo += [m for m in re.findall(r'#include "([^"/]+)"', fh.read())
                     if os.path.exists(os.path.join(csrc, m))]
    assert seen == set(bench.PAIR_KERNEL_SOURCES), seen
    for name in ("PAIR_KERNEL_COUNTERS", "MEASURED_COSTS"):
        v = getattr(bench, name)
        assert v is None or set(v) >= {"sources"}
