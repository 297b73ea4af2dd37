"""Host-side checks of bench.py that need no GPU: the one-GPU contract, the algorithmic flop count of one
apply, and the source digest that ties the committed counter summaries to the HIP sources."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr


def test_f_apply_formula():
    # 8 flops per complex MAC over the pair terms, the exchange and the diagonal (mesh8_ao64: 6.598 TFLOP)
    F = bench.f_apply(512, 64, 4, 8, 256, 8)
    pair = 256 * 64 * (8 ** 2 + 4 ** 2) + 256 ** 2 * 4 ** 2 + 256 * 8 * 4 * 8 * (8 + 4)
    ref = 8 * (512 ** 2 * pair + 2 * 512 * 8 * 4 * 256 * 8 + 256 ** 2 * 8) + 2 * 512 * 32 * 8
    assert F == ref
    assert abs(F / 1e12 - 6.5976) < 1e-3
    # the executed count scales the pair-density and W terms by the formed q; the X term counts every pair
    Fx = bench.f_apply(512, 64, 4, 8, 256, 8, q_formed=260)
    assert F - Fx == 8 * 512 * (512 - 260) * (256 * 64 * (8 ** 2 + 4 ** 2) + 256 ** 2 * 4 ** 2)


def test_source_digest_matches_committed_profiles():
    # the traffic figure is reported only when the committed counter summary was taken on the apply's sources
    dig = bench.source_digest()
    assert len(dig) == 16
    txt = open(os.path.join(ROOT, "profiles", "pmc_wstep_mesh16_ao128_bf16x3.txt")).read()
    assert "source_digest=" in txt
    stored = txt.split("source_digest=")[1].split()[0]
    if stored != dig:
        pytest.skip("the HIP sources changed since the counter summary was taken (traffic is then null)")
    assert stored == dig
