"""amg_spmv_dot_noalloc (static device scratch, no allocation) against
amg_spmv_dot (allocating): the same kernels on the same inputs, so y and the
dot product must agree bit for bit; both against the definition as well.  Two
calls in a row on the GPU, the second with a smaller matrix, so the second
call runs on what the first left in the shared scratch."""
import numpy as np
import pytest

import gen
from gen import fields

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2602_23613_amd as amglib   # noqa: E402

EPS = np.finfo(np.float64).eps


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_noalloc_spmv_dot_matches_allocating_entry_point():
    d = _dev()
    for N, seed in ((24, 11), (6, 12)):
        p = gen.make_problem("hex", N, alpha=lambda m: fields.subdomain_log_uniform(m, 4, seed))
        A = p.A
        n = A.shape[0]
        x = np.random.default_rng(seed).standard_normal(n)
        rp = torch.tensor(A.indptr.astype(np.int64), device=d)
        ci = torch.tensor(A.indices.astype(np.int32), device=d)
        va = torch.tensor(A.data, device=d)
        xt = torch.tensor(x, device=d)
        y_ref = torch.zeros_like(xt)
        d_ref = torch.zeros(1, dtype=torch.float64, device=d)
        amglib.spmv_dot(rp, ci, va, xt, y_ref, d_ref)
        y = torch.full_like(xt, np.nan)
        dot = torch.full((1,), np.nan, dtype=torch.float64, device=d)
        print(f"noalloc spmv_dot: hex {N}^3, n = {n}", flush=True)
        amglib.spmv_dot(rp, ci, va, xt, y, dot, noalloc=True)
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref), N
        assert torch.equal(dot, d_ref), (N, dot.item(), d_ref.item())
        yy = A @ x
        scale = abs(A) @ abs(x)
        assert np.max(np.abs(y.cpu().numpy() - yy) / scale) <= 1e-14
        assert abs(dot.item() - x @ yy) <= n * EPS * (abs(x) @ scale)
