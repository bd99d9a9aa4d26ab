"""Debug mode: the library's bounds check of the connectivity and the slot
maps before each launch.  The faulty inputs are made on the host side of the
check (a node id edited in the device connectivity after the pattern was
built); with the check on, every call reports LFEM_EINVAL naming the element
and launches nothing, so no kernel ever reads through a bad id."""

import pytest
import torch

import meshgen
from gpu_util import order_mesh

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_14035_amd as lf
    return lf


@pytest.fixture
def debug(lf):
    prev = lf.lfem_set_debug(True)
    yield
    lf.lfem_set_debug(prev)


def calls(lf, d):
    """Every entry point that reads the connectivity, as (name, thunk)."""
    N, n_amb = d.N, d.coords.shape[0]
    x = torch.ones(N, dtype=torch.float64, device="cuda")
    nu = torch.ones(n_amb, N, dtype=torch.float64, device="cuda")
    g = torch.empty(n_amb, N, dtype=torch.float64, device="cuda")
    J = torch.empty(1, dtype=torch.float64, device="cuda")
    out = [("assemble", lambda: d.assemble(lf.LFEM_M | lf.LFEM_A)),
           ("assemble staged", lambda: d.assemble(lf.LFEM_M, scatter=lf.LFEM_SCATTER_STAGED)),
           ("load", lambda: d.load(x)),
           ("energy", lambda: lf.lfem_energy(d.handle, x, x, 1.0, x, x, 1.0, J)),
           ("shape_grad", lambda: lf.lfem_shape_grad(d.handle, x, x, 1.0, x, x, 1.0, g)),
           ("dziuk", lambda: d.dziuk_system(0.1)),
           ("autotune", lambda: lf.lfem_pattern_autotune(d.handle, d.pattern, lf.LFEM_M))]
    if d.domain == lf.LFEM_SURFACE:
        out.append(("kll", lambda: d.kll(nu, x)))
    return out


@pytest.mark.parametrize("t", [("surface", 2, 2), ("bulk", 3, 2), ("surface", 1, 1), ("bulk", 3, 3)])
def test_debug_checks(lf, debug, t):
    # the cubic tetrahedra take the 16-bit slot map
    m = order_mesh(*t) if t[2] > 2 else meshgen.small_mesh(*t, size=3)
    d = lf.DeviceMesh.from_dict(m)
    d.build_pattern()
    lf.lfem_set_debug(False)
    ref = d.assemble(lf.LFEM_M | lf.LFEM_A, scatter=lf.LFEM_SCATTER_BLOCKED)
    lf.lfem_set_debug(True)
    # valid input: every call passes the check, results unchanged
    got = d.assemble(lf.LFEM_M | lf.LFEM_A, scatter=lf.LFEM_SCATTER_BLOCKED)
    assert torch.equal(got["M"], ref["M"]) and torch.equal(got["A"], ref["A"])
    for name, fn in calls(lf, d):
        fn()
    # the autotune call may have rebuilt the block schedule (for tetrahedra
    # the colour order, and with it the bits, follow the schedule)
    ref = d.assemble(lf.LFEM_M | lf.LFEM_A, scatter=lf.LFEM_SCATTER_BLOCKED)
    torch.cuda.synchronize()
    e = min(5, d.T - 1)
    saved = d.conn[0, e].item()
    # a node id out of range: every call fails before launching
    d.conn[0, e] = d.N + 7
    torch.cuda.synchronize()
    for name, fn in calls(lf, d):
        with pytest.raises(lf.LfemError) as ei:
            fn()
        assert ei.value.status == lf.LFEM_EINVAL, name
        assert f"element {e}:" in str(ei.value) and "outside [0, N)" in str(ei.value), (name, str(ei.value))
    # an id in range but not the one the pattern was built with: the
    # pattern-based calls fail on the slot check
    far = int((saved + d.N // 2) % d.N)
    d.conn[0, e] = far
    torch.cuda.synchronize()
    with pytest.raises(lf.LfemError) as ei:
        d.assemble(lf.LFEM_M | lf.LFEM_A)
    assert ei.value.status == lf.LFEM_EINVAL and f"element {e}:" in str(ei.value), str(ei.value)
    assert "slot" in str(ei.value)
    # a batch holding the mesh is checked at creation and at every run
    with pytest.raises(lf.LfemError) as ei:
        lf.lfem_batch_create([d.handle], [d.pattern], lf.LFEM_M)
    assert ei.value.status == lf.LFEM_EINVAL
    d.conn[0, e] = saved
    torch.cuda.synchronize()
    b = lf.lfem_batch_create([d.handle], [d.pattern], lf.LFEM_M)
    v = torch.empty(d.nnz, dtype=torch.float64, device="cuda")
    lf.lfem_assemble_batch(b, [v])
    # the batch runs the scatter the autotune call above chose
    assert torch.equal(v, d.assemble(lf.LFEM_M)["M"])
    d.conn[0, e] = d.N
    torch.cuda.synchronize()
    with pytest.raises(lf.LfemError) as ei:
        lf.lfem_assemble_batch(b, [v])
    assert ei.value.status == lf.LFEM_EINVAL
    d.conn[0, e] = saved
    torch.cuda.synchronize()
    lf.lfem_batch_destroy(b)
    # restored: valid again
    got = d.assemble(lf.LFEM_M | lf.LFEM_A, scatter=lf.LFEM_SCATTER_BLOCKED)
    assert torch.equal(got["M"], ref["M"]) and torch.equal(got["A"], ref["A"])
    d.close()


def test_debug_flag_round_trip(lf):
    prev = lf.lfem_set_debug(True)
    assert lf.lfem_set_debug(False) is True
    assert lf.lfem_set_debug(prev) is False
