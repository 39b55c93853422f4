"""CPU: the host side of bench.py -- the region sizes and algorithmic bytes
the roofline divides by, and the refusal of several GPUs.

The regions of a subdomain (Sec. 3.1.2: the padded field, here the sites a
hop stage must produce) are L1 balls around the subdomain box restricted to
one parity.  Their sizes have a closed form, independent of the site-by-site
enumeration in bench.region_counts: with V the box volume and, over the
partitioned dimensions only, S1 = sum of the box's face areas (prod of the
other three extents) and S2 = sum over pairs of the products of the two
remaining extents, the sites at L1 distance 1 are 2 S1 and at distance 2 are
2 S1 (two layers out along one axis) + 4 S2 (one step along each of two
axes); with even extents every layer is half even, half odd.  So
C = V/2, N1 = V/2 + S1, N2 = V/2 + S1 + S1 + 2 S2.
"""
import itertools
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from workloads.configs import CONFIGS  # noqa: E402


def closed_form_regions(sub, dims):
    part = [m for m in range(4) if sub[m] < dims[m]]
    V = int(np.prod(sub))
    S1 = sum(int(np.prod([sub[n] for n in range(4) if n != m])) for m in part)
    S2 = sum(int(np.prod([sub[k] for k in range(4) if k not in (m, n)])) for m, n in itertools.combinations(part, 2))
    return V // 2, V // 2 + S1, V // 2 + 2 * S1 + 2 * S2


@pytest.mark.parametrize("sub,dims", [
    ((4, 4, 4, 8), (16, 16, 16, 32)),    # 16^3x32 workload
    ((8, 8, 8, 16), (32, 32, 32, 64)),   # 32^3x64 workload
    ((4, 4, 4, 4), (8, 8, 8, 8)),
    ((4, 4, 4, 2), (8, 8, 4, 2)),        # two dimensions not partitioned
    ((6, 6, 6, 12), (24, 24, 24, 48)),
])
def test_region_counts_match_the_closed_form(sub, dims):
    assert bench.region_counts(sub, dims) == closed_form_regions(sub, dims)


def test_region_sizes_of_the_workloads():
    assert bench.region_counts(CONFIGS["c2"].sub, CONFIGS["c2"].dims) == (256, 704, 1440)
    assert bench.region_counts(CONFIGS["c4"].sub, CONFIGS["c4"].dims) == (4096, 7680, 12416)


def test_algorithmic_bytes_of_the_dominant_stage():
    """h2 (N2 <- N1 with the centre field on C), FP16 storage: every input
    site read once (N1 and C: 48 bytes of halves + a 4-byte scale per 5D
    site), every output site written once (N2), and the 8 links of every
    output 4D site once in FP16 (8 x 18 x 2 bytes), over all subdomains."""
    for name, expect in (("c2", 489_553_920), ("c4", 4_779_933_696)):
        cfg = CONFIGS[name]
        nC, nN1, nN2 = closed_form_regions(cfg.sub, cfg.dims)
        ns = cfg.n_subdomains
        by_hand = ns * cfg.Ls * 52 * (nN1 + nC + nN2) + ns * 8 * 18 * 2 * nN2
        got, _ = bench.stage_bytes(cfg, "fp16")
        assert got[12] == by_hand == expect


def test_outer_hop_bytes():
    """Outer FP32 hops: 96 bytes per 5D spinor site, 8 FP32 links (8 x 18 x 4
    bytes) per output 4D site; hop 1 and 3 read one field and write one, hop 2
    also reads the centre field, hop 4 the centre field and the dot's field."""
    cfg = CONFIGS["c4"]
    vh = int(np.prod(cfg.dims)) // 2
    n5 = vh * cfg.Ls
    got, _ = bench.stage_bytes(cfg, "fp16")
    links = vh * 8 * 18 * 4
    assert got[21] == got[23] == 2 * 96 * n5 + links
    assert got[22] == 3 * 96 * n5 + links
    assert got[24] == 4 * 96 * n5 + links


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
