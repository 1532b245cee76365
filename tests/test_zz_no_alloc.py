"""The allocation-free contact factor (sph_contact_factor_noalloc), through the
C ABI, against sph_contact_factor on the same solver state: per solid
particle bit for bit, per-body means within 1e-13 relative (device
compensated sums in a fixed order against the host's compensated sums in
the caller's order).  Two calls in a row on different solvers, the second
smaller, share the library's static scratch."""
import sys

import numpy as np
import pytest

from paper_2512_09904_amd import cases

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def sph():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_09904_amd import sph as S
    S.lib()
    return S


def _compare(sph, case, precision, steps):
    import torch
    s = sph.Solver(case, precision=precision)
    if steps:
        s.step(steps)
        s.reduce()
    z_host, m_host = s.contact_factor()
    dev = torch.device("cuda", torch.cuda.current_device())
    z = torch.full((case.ns,), float("nan"), dtype=torch.float64, device=dev)
    m = torch.full((len(case.bodies),), float("nan"), dtype=torch.float64, device=dev)
    s.contact_factor_noalloc(z, m)
    s.stream.synchronize()
    zg, mg = z.cpu().numpy(), m.cpu().numpy()
    # the solve is unchanged by either call: the next step's build is the same
    r = s.reduce()
    s.close()
    say("no-alloc contact factor", precision, case.ns, "means", mg, m_host)
    assert np.array_equal(zg, z_host)
    assert np.allclose(mg, m_host, rtol=1e-13, atol=0)
    assert r["flags"] == 0
    return mg


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_noalloc_contact_factor_equals_the_allocating_call(sph, precision):
    big = cases.tank_c1(seed=1)
    small = cases.tank_c1(seed=2, dp=2.5e-3)
    assert small.ns < big.ns and small.nf < big.nf
    _compare(sph, big, precision, 3)
    _compare(sph, small, precision, 0)


def test_noalloc_contact_factor_rejects_bad_calls(sph):
    c = cases.tank_c1(seed=3)
    s = sph.Solver(c)
    with pytest.raises(ValueError):
        s.contact_factor_noalloc(np.zeros(c.ns), None)
    # NULL outputs: only the sort and build run
    s.contact_factor_noalloc(None, None)
    s.step(1)
    assert s.reduce()["flags"] == 0
    s.close()
