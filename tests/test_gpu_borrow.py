"""amg_options.borrow_a: with a device A the hierarchy reads the caller's
arrays in place instead of copying them.  Everything it computes must equal
the copying hierarchy bit for bit; a numeric re-setup from another device A
(same pattern) borrows that one instead, and the V-cycles captured before
must not keep reading the first A."""
import numpy as np
import pytest

import gen
from gen import fields

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2602_23613_amd as amglib   # noqa: E402


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def device_csr(A, d):
    A = A.tocsr()
    return (torch.tensor(A.indptr.astype(np.int64), device=d),
            torch.tensor(A.indices.astype(np.int32), device=d),
            torch.tensor(A.data.astype(np.float64), device=d), A.shape[0], A.shape[1])


@pytest.mark.parametrize("mode", ["blocks", "patch"])
def test_borrowed_a_equals_copied_a(mode):
    d = dev()
    p = gen.make_problem("hex", 10, beta=1.0, alpha=lambda m: fields.subdomain_log_uniform(m, 4, 9),
                         f=lambda n: fields.rhs_uniform(n, 91))
    q = gen.make_problem("hex", 10, beta=1.0, alpha=lambda m: fields.subdomain_log_uniform(m, 4, 10),
                         f=lambda n: fields.rhs_uniform(n, 92))
    Ad, Gd = device_csr(p.A, d), device_csr(p.G, d)
    Hb = amglib.Hierarchy(Ad, Gd, ext_mode=mode, borrow_a=True)
    Hc = amglib.Hierarchy(Ad, Gd, ext_mode=mode)
    f = torch.tensor(p.f, device=d)
    for H in (Hb, Hc):
        assert len(H.info()) > 2
    zb, zc = torch.zeros_like(f), torch.zeros_like(f)
    Hb.vcycle(f, zb)
    Hc.vcycle(f, zc)
    torch.cuda.synchronize()
    assert torch.equal(zb, zc)
    ub, uc = torch.zeros_like(f), torch.zeros_like(f)
    sb, sc = Hb.pcg(f, ub), Hc.pcg(f, uc)
    assert sb["iterations"] == sc["iterations"] and torch.equal(ub, uc)
    # numeric re-setup from a second device A with the same pattern: the
    # borrowing hierarchy switches to it (its earlier graphs are dropped)
    Bd = device_csr(q.A, d)
    assert torch.equal(Bd[0], Ad[0]) and torch.equal(Bd[1], Ad[1])
    Hb.resetup(Bd)
    Hc.resetup(Bd)
    Hf = amglib.Hierarchy(Bd, Gd, ext_mode=mode)
    g = torch.tensor(q.f, device=d)
    zb, zc, zf = torch.zeros_like(g), torch.zeros_like(g), torch.zeros_like(g)
    Hb.vcycle(g, zb)
    Hc.vcycle(g, zc)
    Hf.vcycle(g, zf)
    torch.cuda.synchronize()
    assert torch.equal(zb, zc) and torch.equal(zb, zf)
    # the first A may now change: the borrowing hierarchy no longer reads it
    Ad[2].zero_()
    zb2 = torch.zeros_like(g)
    Hb.vcycle(g, zb2)
    torch.cuda.synchronize()
    assert torch.equal(zb2, zb)
    for H in (Hb, Hc, Hf):
        H.close()


def test_borrowing_hierarchy_rejects_a_host_resetup():
    d = dev()
    p = gen.make_problem("hex", 6, beta=1.0)
    Ad, Gd = device_csr(p.A, d), device_csr(p.G, d)
    H = amglib.Hierarchy(Ad, Gd, borrow_a=True)
    with pytest.raises(amglib.AmgError) as e:
        H.resetup(p.A)
    assert e.value.status == -1
    H.close()
