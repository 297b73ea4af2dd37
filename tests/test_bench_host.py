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


@pytest.mark.parametrize("dims,total", [
    ((64, 16, 4, 4, 64, 3), 4.030e9),            # 4x4x4 mesh, N_ao 16, 4 + 4 bands, N_aux 64, 3 vectors
    ((512, 64, 4, 8, 256, 4), 5.773e12),         # 8x8x8 mesh, LOBPCG block of 4
    ((1728, 96, 6, 10, 384, 8), 317.02e12),      # 12x12x12 mesh, N_ao 96, 6 + 10 bands, N_aux 384
    ((4096, 128, 8, 8, 512, 16), 4503.6e12),     # 16x16x16 mesh, N_ao 128, 8 + 8 bands, N_aux 512, 16 vectors
])
def test_f_apply_at_the_workloads(dims, total):
    # the algorithmic count of one apply at each workload (the GFLOP/s of every record divides it by time)
    assert abs(bench.f_apply(*dims) / total - 1) < 2e-4


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


def test_roofline_counts_of_the_fused_w_step():
    # the dominant kernel at 16^3 (W step with the direct blocks, P on chip): its algorithmic flops per pair
    # are the W term plus the direct-block term, and its bytes per launch read G_v and M_c once, W(q) once per
    # q of the batch and write T once (16 q x 4096 k pairs per full batch)
    from types import SimpleNamespace
    p = SimpleNamespace(n_aux=512, n_ao=128, nv=8, nc=8, Nk=4096)
    f = bench.kernel_flops_per_pair(p, "bf16x3", "fused")
    assert f["wstep"] == 8 * 512 ** 2 * 64 + 8 * 512 * 64 * 64 == 150994944
    assert "dblock" not in f
    assert f["pairdens_v"] == f["pairdens_c"] == 8 * 512 * 128 * 64
    b = bench.kernel_bytes_per_pair(p, "bf16x3", "fused")
    per_pair = 8 * (64 * 512 + 64 * 512) + 8 * 512 * 512 / 4096 + 8 * 64 * 64
    assert b["wstep"] == per_pair
    assert abs(16 * 4096 * per_pair / 1e9 - 36.54) < 0.01
    # the bench's per-launch figure averages over 128 batches of 16 q and one of 4 (65,155 pairs)
    assert abs(2052 * 4096 / 129 * per_pair / 1e9 - 36.33) < 0.01
    # the B_c route prices the conduction side at its own executed count (about twice the M_cc' count)
    q = SimpleNamespace(n_aux=256, n_ao=64, nv=4, nc=8, Nk=512)
    u = bench.kernel_flops_per_pair(q, "bf16x3", "u")["dblock"]
    mc = bench.kernel_flops_per_pair(q, "bf16x3", "mc")
    assert u == 8 * 8 * 64 * 256 * 16 + 8 * 64 * 64 * 16
    assert 2.0 < u / (mc["pairdens_c"]) < 2.1
