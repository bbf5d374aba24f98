"""GPU test of adr_precompute_phi_noalloc, the matrix-function precompute that
allocates no device memory (its work area is a fixed array in each GPU's
memory), against adr_precompute_phi, which works in a block the library
allocates.  Both run the same kernels in the same order, so the results must
agree bitwise (the FP64 parity gate of 1e-12 is checked too).  Two calls in a
row, the second with a smaller matrix, exercise the reuse of the fixed array,
which keeps the previous call's contents."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _operator(dev, n, diff, vel):
    A, _ = dev.adr_build_1d_ops(n, 0.0, 1.0, diff, vel)
    return dev.to_device_f64(A)


def test_noalloc_matches_allocating_precompute(dev):
    import torch
    # a stiff advective operator at the largest size the fixed array takes, then
    # a smaller diffusion-only one (the second call reuses the array)
    for n, diff, vel, tau in ((dev.ADR_PHI_NOALLOC_MAX_N, 5e-3, 0.1, 5e-3), (300, 5e-3, 0.1, 5e-3),
                              (97, 1.0, 0.0, 1e-3)):
        A = _operator(dev, n, diff, vel)
        ref = dev.adr_precompute_phi(A, tau)
        got = dev.adr_precompute_phi_noalloc(A, tau)
        torch.cuda.synchronize()
        for j, (r, g) in enumerate(zip(ref, got)):
            r, g = r.cpu().numpy(), g.cpu().numpy()
            rel = np.abs(g - r).max() / np.abs(r).max()
            print(f"n={n} matrix {j}: max rel diff {rel:.1e}")
            assert rel <= 1e-12
            assert np.array_equal(g, r)


def test_noalloc_partial_outputs_and_limit(dev):
    import torch
    n = 64
    A = _operator(dev, n, 1.0, 0.3)
    E, P1, P2 = dev.adr_precompute_phi(A, 2e-3)
    P1b = torch.full((n * n,), float("nan"), dtype=torch.float64, device="cuda")
    _, got, _ = dev.adr_precompute_phi_noalloc(A, 2e-3, P1=P1b, want=(False, True, False))
    torch.cuda.synchronize()
    assert torch.equal(got, P1)
    big = _operator(dev, dev.ADR_PHI_NOALLOC_MAX_N + 1, 1.0, 0.0)
    with pytest.raises(dev.AdrError) as ei:
        dev.adr_precompute_phi_noalloc(big, 1e-3)
    assert ei.value.status == dev.ADR_ENOMEM
