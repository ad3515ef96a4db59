"""Launch batching: kernels with one workgroup per row, block or column go out
in batches of at most 2^22 workgroups, because a dispatch counts its
work-items in 32 bits (at 256 threads per workgroup, 16.8M rows would
already overflow it).  HCURL_AMG_MAX_WG lowers the batch size, so a small
problem runs every batched launch in many pieces.  The batch boundaries do
not change any row's arithmetic, so the hierarchy (every A_l and P_l), one
V-cycle and PCG must match the default launch bit for bit.

The batched run happens in a child process (the batch size is read once per
process); both processes use the one GPU in turn."""
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

import gen
from gen import fields

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2602_23613_amd as amglib   # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent("""
    import sys, numpy as np, torch
    sys.path.insert(0, {root!r})
    import gen, paper_2602_23613_amd as amglib
    from gen import fields
    out = {{}}
    for mode in ("patch", "blocks"):
        p = gen.make_problem("hex", 10, beta=1.0,
                             alpha=lambda m: fields.subdomain_log_uniform(m, 4, 7),
                             f=lambda n: fields.rhs_uniform(n, 77))
        H = amglib.Hierarchy(p.A, p.G, ext_mode=mode)
        for l in range(len(H.info())):
            A, P = H.level(l)
            out[f"{{mode}}_A{{l}}"] = A.data
            if P is not None:
                out[f"{{mode}}_P{{l}}"] = P.data
        f = torch.from_numpy(p.f).cuda()
        z = torch.zeros_like(f)
        H.vcycle(f, z)
        out[f"{{mode}}_z"] = z.cpu().numpy()
        u = torch.zeros_like(f)
        st = H.pcg(f, u, rtol=1e-8, maxit=200)
        out[f"{{mode}}_u"] = u.cpu().numpy()
        out[f"{{mode}}_its"] = np.array([st["iterations"]])
        H.close()
    np.savez({path!r}, **out)
    print("child done", flush=True)
""")


def run(mode, p):
    H = amglib.Hierarchy(p.A, p.G, ext_mode=mode)
    out = {}
    for l in range(len(H.info())):
        A, P = H.level(l)
        out[f"{mode}_A{l}"] = A.data
        if P is not None:
            out[f"{mode}_P{l}"] = P.data
    f = torch.from_numpy(p.f).cuda()
    z = torch.zeros_like(f)
    H.vcycle(f, z)
    out[f"{mode}_z"] = z.cpu().numpy()
    u = torch.zeros_like(f)
    st = H.pcg(f, u, rtol=1e-8, maxit=200)
    out[f"{mode}_u"] = u.cpu().numpy()
    out[f"{mode}_its"] = np.array([st["iterations"]])
    H.close()
    return out


def test_batched_launches_match_single_launches(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    path = str(tmp_path / "batched.npz")
    env = dict(os.environ, HCURL_AMG_MAX_WG="3")
    print("child: hex 10^3, HCURL_AMG_MAX_WG=3", flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, path=path)], env=env,
                       cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    got = dict(np.load(path))
    p = gen.make_problem("hex", 10, beta=1.0, alpha=lambda m: fields.subdomain_log_uniform(m, 4, 7),
                         f=lambda n: fields.rhs_uniform(n, 77))
    ref = {}
    for mode in ("patch", "blocks"):
        ref.update(run(mode, p))
    assert sorted(got) == sorted(ref)
    for k in ref:
        assert np.array_equal(got[k], ref[k]), k
