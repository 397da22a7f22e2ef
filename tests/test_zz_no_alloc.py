"""The allocation-free operator apply (ls_apply_A_noalloc) against ls_apply_A
through the C ABI: two calls in a row on one handle (the second with a
smaller batch), both precisions, then a handle on a smaller grid; the
results must equal the allocating entry point's bit for bit (the same
kernels on the same inputs). Batches beyond the static scratch are refused
on the host with the limit in the message."""
import ctypes
import math

import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _pair(lib, s, x, precision):
    y_ref = torch.empty_like(x)
    y_na = torch.full_like(x, float("nan"))
    nb = x.shape[0]
    assert lib.ls_apply_A(s._h, x.data_ptr(), nb, y_ref.data_ptr(), precision) == 0, lib.ls_last_error()
    st = lib.ls_apply_A_noalloc(s._h, x.data_ptr(), nb, y_na.data_ptr(), precision)
    assert st == 0, lib.ls_last_error()
    return y_ref.cpu().numpy(), y_na.cpu().numpy()


def test_noalloc_apply_matches_allocating_apply():
    from paper_1705_09443_amd import LSSolver, _lib
    lib = _lib.load()
    rng = np.random.default_rng(3)
    for n, nbs in ((255, (3, 1)), (63, (5, 2))):
        omega = 2 * math.pi * (n + 1) / 16.0
        m = workloads.gaussian_bump_medium(n, 2, 8, (0.2, 0.8), (0.02, 0.05), (-0.4, 0.4), seed=n)
        with LSSolver(torch.as_tensor(m).cuda(), omega, 12, 4, precision="mixed") as s:
            for nb in nbs:
                xr = rng.standard_normal((nb, n, n)) + 1j * rng.standard_normal((nb, n, n))
                for prec, dt in ((_lib.LS_FP64, torch.complex128), (_lib.LS_MIXED, torch.complex64)):
                    x = torch.as_tensor(xr).to(device="cuda", dtype=dt)
                    y_ref, y_na = _pair(lib, s, x, prec)
                    assert np.array_equal(y_ref, y_na), (n, nb, prec, np.abs(y_ref - y_na).max())
                    print(f"[noalloc] n={n} nrhs={nb} precision={prec}: identical to ls_apply_A", flush=True)


def test_noalloc_refuses_batches_beyond_the_scratch():
    from paper_1705_09443_amd import LSSolver, _lib
    lib = _lib.load()
    n = 1023
    omega = 2 * math.pi * 64.0
    m = np.zeros((n, n))
    with LSSolver(torch.as_tensor(m).cuda(), omega, 12, 4, precision="mixed") as s:
        x = torch.zeros((5, n, n), dtype=torch.complex64, device="cuda")
        y = torch.empty_like(x)
        # 2048 x 1024 x 8 B = 16.0 MiB per right-hand side (rows padded to 1024): 4 fit in 64 MiB, 5 do not
        st = lib.ls_apply_A_noalloc(s._h, x.data_ptr(), 5, y.data_ptr(), _lib.LS_MIXED)
        assert st == _lib.LS_E_INVALID
        msg = lib.ls_last_error().decode()
        assert "at most 4" in msg, msg
        x64 = torch.zeros((3, n, n), dtype=torch.complex128, device="cuda")
        y64 = torch.empty_like(x64)
        st = lib.ls_apply_A_noalloc(s._h, x64.data_ptr(), 3, y64.data_ptr(), _lib.LS_FP64)
        assert st == _lib.LS_E_INVALID and "at most 2" in lib.ls_last_error().decode()
        st = lib.ls_apply_A_noalloc(s._h, x.data_ptr(), 4, y.data_ptr(), _lib.LS_MIXED)
        assert st == 0, lib.ls_last_error()
        assert float(y[:4].abs().max()) == 0.0   # m = 0: A = I on a zero field
