"""GPU parity of the FFT operator at every transform length the library
instantiates at compile time (P = 128 ... 2048 here; 4096 is the largest-grid
test's), with grids whose row count is not a multiple of the sequences per
workgroup, so the last row group is partly empty. The oracle is the dense
operator of eq. LS_d_c by numpy FFT; A and K (no medium factor) are both
checked, in float64 (1e-13, round-off of length-P transforms) and complex64
(2e-6)."""
import sys

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# n: transform length P = 2^k >= 2(n + 1); n mod 8 (P <= 1024) or n mod 4
# (P = 2048) leaves the last group of rows partly empty
@pytest.mark.parametrize("n", [70, 129, 300, 701])
def test_apply_A_and_K_per_length(n):
    from paper_1705_09443_amd import LSSolver
    omega = 2 * np.pi * 6.0
    m = workloads.gaussian_bump_medium(n, 2, 6, (0.2, 0.8), (0.04, 0.1), (-0.4, 0.4), seed=11)
    op = oracle.DenseOperator(2, n, omega, m)
    rng = np.random.default_rng(n)
    x = rng.standard_normal((3, n, n)) + 1j * rng.standard_normal((3, n, n))
    wantA = np.stack([op.apply_A(x[j]) for j in range(3)])
    wantK = np.stack([op.apply_K(x[j]) for j in range(3)])
    say(f"[fft n={n}] GPU setup and applies")
    with LSSolver(torch.as_tensor(m).cuda(), omega, 12, 4, precision="fp64") as s:
        xd = torch.as_tensor(x).cuda()
        yA = s.apply_A(xd).cpu().numpy()
        yK = s.apply_K(xd).cpu().numpy()
        yA32 = s.apply_A(xd.to(torch.complex64), "mixed").cpu().numpy()
        yK32 = s.apply_K(xd.to(torch.complex64), "mixed").cpu().numpy()
    eA, eK, eA32, eK32 = rel(yA, wantA), rel(yK, wantK), rel(yA32, wantA), rel(yK32, wantK)
    say(f"[fft n={n}] A {eA:.2e} K {eK:.2e} A c64 {eA32:.2e} K c64 {eK32:.2e}")
    assert eA <= 1e-13 and eK <= 1e-13
    assert eA32 <= 2e-6 and eK32 <= 2e-6
