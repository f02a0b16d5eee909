"""Plans on different streams: device blocks freed by one plan are reused by the next on
another stream (after a wait on the freeing stream), and every solve gives the same bits
as a plan on the default stream."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1408_3048_amd import Plan  # noqa: E402

from gpu_common import problem  # noqa: E402


def test_plans_alternating_streams_equal_default_stream():
    sc, pr = problem("small_iqu")
    b_host = pr.rhs(pr.signal(sc.sky) + sc.noise)
    pl = Plan.from_scan(sc, precision="mixed", coarse=True)
    x_ref, i_ref = pl.pcg_solve(torch.from_numpy(b_host).cuda(), precond="2lvl",
                                precision="mixed", tol=1e-9, max_iter=3000)
    torch.cuda.synchronize()
    pl.close()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for s in (s1, s2, s1, s2):
        with torch.cuda.stream(s):
            p = Plan.from_scan(sc, precision="mixed", coarse=True)
            b = torch.from_numpy(b_host).cuda()
            x, info = p.pcg_solve(b, precond="2lvl", precision="mixed", tol=1e-9, max_iter=3000)
            s.synchronize()
            assert info["iterations"] == i_ref["iterations"]
            assert torch.equal(x, x_ref)
            p.close()
    torch.cuda.synchronize()
