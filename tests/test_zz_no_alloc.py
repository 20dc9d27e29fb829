"""kog_sweep_batch_noalloc (the sweep whose workspace is a static device array, for
callers that cannot allocate) against kog_sweep_batch with a caller workspace, through
the C ABI: G, U, V, sigma and the sweep counts bit for bit, on two calls in a row, the
second with a smaller batch (the scratch keeps the first call's contents), in both
persistent and plain modes, both precisions; a batch whose workspace exceeds the
scratch is refused before any device work."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _mats(rng, ns, dtype):
    return [np.asfortranarray((rng.standard_normal((n, n)) *
                               np.exp2(rng.integers(-8, 9, (n, n)))).astype(dtype)) for n in ns]


def _call(L, fn, p, mode, ordering, ws=None):
    import torch

    from paper_2407_13116_amd import sweep as sw

    G = p.G.clone()
    U, V = torch.empty_like(G), torch.empty_like(G)
    sigma = torch.empty(int(p.n.sum()), dtype=G.dtype, device=G.device)
    sweeps = torch.empty(len(p.n), dtype=torch.int32, device=G.device)
    n = np.ascontiguousarray(p.n)
    off = np.ascontiguousarray(p.off)
    dt = 1 if G.dtype == torch.float64 else 0
    common = (dt, len(n), n.ctypes.data_as(ctypes.c_void_p), off.ctypes.data_as(ctypes.c_void_p),
              G.data_ptr(), U.data_ptr(), V.data_ptr(), sigma.data_ptr(), sweeps.data_ptr(), 12,
              1.0, 0, mode, ordering)
    st = torch.cuda.current_stream().cuda_stream or None
    if fn == "noalloc":
        rc = L.kog_sweep_batch_noalloc(*common, st)
    else:
        need = sw.workspace_bytes(G.dtype, p.n)
        ws = torch.empty(need, dtype=torch.uint8, device=G.device)
        rc = L.kog_sweep_batch(*common, ws.data_ptr(), need, st)
    assert rc == 0, L.ksvd2_last_error()
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (G, U, V, sigma, sweeps)]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("mode", [1, 0])
def test_noalloc_matches_workspace_entry(dtype, mode):
    from paper_2407_13116_amd import _lib
    from paper_2407_13116_amd import sweep as sw

    L = _lib.lib()
    rng = np.random.default_rng(41 + mode)
    # first call: orders past 256 (their two-step passes go through the second buffer)
    big = [300, 16, 2, 130, 64, 258, 8, 200, 34, 100, 6, 272]
    small = [40, 4, 18, 2, 66]
    for ns in (big, small):
        p = sw.Packed(_mats(rng, ns, dtype), dtype=dtype)
        for ordering in (1, 0):
            want = _call(L, "ws", p, mode, ordering)
            got = _call(L, "noalloc", p, mode, ordering)
            for a, b, name in zip(got, want, ("G", "U", "V", "sigma", "sweeps")):
                assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), (ns, ordering, name)
            assert np.all(got[4] != 0)


def test_noalloc_refuses_oversized_batch_and_graph_mode():
    import torch

    from paper_2407_13116_amd import _lib
    L = _lib.lib()
    # forty FP64 matrices of order 512 under the modified modulus ordering in the
    # persistent mode: their two-step passes need an 80 MiB second buffer, more than the
    # 64 MiB scratch
    k, nn = 40, 512
    n = np.full(k, nn, dtype=np.int32)
    off = (np.arange(k, dtype=np.int64) * nn * nn)
    G = torch.zeros(k * nn * nn, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream or None
    args = (1, k, n.ctypes.data_as(ctypes.c_void_p), off.ctypes.data_as(ctypes.c_void_p),
            G.data_ptr(), G.data_ptr(), G.data_ptr(), None, None, 1, 1.0, 0)
    assert L.kog_sweep_batch_noalloc(*args, 1, 1, st) == -4
    assert b"kog_sweep_batch" in L.ksvd2_last_error()
    assert L.kog_sweep_batch_noalloc(*args, 2, 1, st) == -1
    torch.cuda.synchronize()
    assert torch.count_nonzero(G).item() == 0          # nothing ran
