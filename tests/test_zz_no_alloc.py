"""The allocation-free entry point mm_gemm_tn_f64_noalloc against mm_gemm_tn_f64 (the
same product E = Z^T (AZ) with per-call partials), through the C-ABI: bitwise equal
results on consecutive calls of decreasing size (the fixed scratch keeps the previous
call's partials), one of them filling the whole scratch, and the size limit rejected on
the host before any launch."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1408_3048_amd as pkg  # noqa: E402
from paper_1408_3048_amd import _lib as L  # noqa: E402


def _pair(n, ra, rb, seed):
    rng = np.random.default_rng(seed)
    A = torch.from_numpy(rng.standard_normal((n, ra))).cuda()
    B = torch.from_numpy(rng.standard_normal((n, rb))).cuda()
    return A, B


@pytest.mark.parametrize("shapes", [[(4000, 48, 32), (1000, 32, 16)],
                                    [(256, 1024, 1024), (4096, 64, 48)]])
def test_noalloc_matches_allocating_entry_point(shapes):
    for k, (n, ra, rb) in enumerate(shapes):
        print(f"[noalloc] call {k}: n={n} ra={ra} rb={rb}", flush=True)
        A, B = _pair(n, ra, rb, seed=100 + k)
        ref = L.gemm_tn_f64(A, B)
        C = torch.full((ra, rb), float("nan"), dtype=torch.float64, device="cuda")
        L.gemm_tn_f64_noalloc(A, B, C)
        torch.cuda.synchronize()
        assert torch.equal(C, ref), (k, float((C - ref).abs().max()))
        exact = A.cpu().numpy().T @ B.cpu().numpy()
        assert np.max(np.abs(C.cpu().numpy() - exact)) <= 1e-12 * np.max(np.abs(exact))


def test_noalloc_rejects_partials_beyond_the_scratch():
    A, B = _pair(4, 1040, 1040, seed=7)
    C = torch.zeros((1040, 1040), dtype=torch.float64, device="cuda")
    with pytest.raises(pkg.MMError) as e:
        L.gemm_tn_f64_noalloc(A, B, C)
    assert e.value.status == pkg.MM_ERR_ARG and "scratch" in str(e.value)
    assert torch.count_nonzero(C) == 0
