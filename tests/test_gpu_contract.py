"""The boundary's contract on the GPU: calls that only enqueue can be
recorded into a graph and replayed; one handle per stream; argument errors
are raised before anything is launched."""
import numpy as np
import pytest
import torch

import smk_inputs as si

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mr():
    import paper_2605_30379_amd as m
    assert torch.cuda.is_available()
    m.lib()
    return m


def _replays_match(g, outs, eager, busy):
    """Replay g several times with eager work and synchronisations between
    the replays; every replay must reproduce the eager results bit for bit."""
    for r in range(4):
        for o in outs:
            o.fill_(float("nan"))
        busy()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            assert torch.equal(o, e), f"replay {r} differs"


def test_functionals_replay_from_a_graph(mr):
    """first_entrance, reliability and availability recorded on a side stream
    (the host masks and initial law travel as kernel arguments), replayed."""
    d, n = 6, 3000
    k = si.weibull_kernel(d, n, 61, device="cuda")
    q = k.q
    up = [1, 1, 1, 0, 0, 0]
    alpha = np.eye(d)[0]
    inD = [0, 0, 0, 0, 0, 1]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        psi = mr.psi_inverse(q)
        P = mr.transition(psi, q)
        eager = [*mr.first_entrance(q, inD, alpha), mr.reliability(q, up, alpha), mr.availability(P, up, alpha)]
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            gF = mr.first_entrance(q, inD, alpha)
            gR = mr.reliability(q, up, alpha)
            gA = mr.availability(P, up, alpha)
    torch.cuda.synchronize()
    other = si.weibull_kernel(d, n, 62, device="cuda").q

    def busy():
        # eager calls on the default stream with other masks and laws in between
        mr.first_entrance(other, [1, 0, 0, 0, 0, 0], np.eye(d)[3])
        mr.availability(mr.transition(mr.psi_inverse(other), other), [0, 0, 0, 1, 1, 1], np.eye(d)[4])

    _replays_match(g, [gF[0], gF[1], gR, gA], eager, busy)
    mr.sync_status()


def test_batched_launch_replays_from_a_graph(mr):
    work = [(3, 700), (9, 1500), (17, 1024), (5, 40)]
    qs = [si.weibull_kernel(d, n, 70 + i, device="cuda").q for i, (d, n) in enumerate(work)]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan = mr.BatchedPlan(qs, "mixed")
        eager = [o.clone() for o in plan.launch()]
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            outs = plan.launch()
    torch.cuda.synchronize()
    singles = [mr.psi_inverse(q, "mixed") for q in qs]
    for e, o in zip(eager, singles):
        assert torch.equal(e, o)          # batched equals single calls, bit for bit

    def busy():
        mr.psi_inverse_batched([q * 0.5 for q in qs[:2]], "fp64")

    _replays_match(g, outs, eager, busy)
    # A plan prepared later on the same stream retires the first one.
    with torch.cuda.stream(s):
        mr.BatchedPlan(qs[:1], "fp64")
        with pytest.raises(mr.MrinvError):
            plan.launch()
    torch.cuda.synchronize()


def test_one_handle_per_stream(mr):
    """Two streams run availability (which uses the handle's scratch) on
    different problems at the same time; each result equals its serial one."""
    d, n = 8, 20000
    qa = si.weibull_kernel(d, n, 81, device="cuda").q
    qb = si.lognormal_kernel(d, n, 82, device="cuda").q
    up = [1] * 4 + [0] * 4
    Pa = mr.transition(mr.psi_inverse(qa), qa)
    Pb = mr.transition(mr.psi_inverse(qb), qb)
    ra = mr.availability(Pa, up, np.eye(d)[0])
    rb = mr.availability(Pb, up, np.eye(d)[2])
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    outs = []
    for _ in range(3):
        with torch.cuda.stream(s1):
            xa = mr.availability(Pa, up, np.eye(d)[0])
        with torch.cuda.stream(s2):
            xb = mr.availability(Pb, up, np.eye(d)[2])
        outs.append((xa, xb))
    torch.cuda.synchronize()
    for xa, xb in outs:
        assert torch.equal(xa, ra) and torch.equal(xb, rb)


def test_mismatched_horizons_are_rejected_before_launch(mr):
    """Every operand of a call must have the horizon of psi (and be square where
    the operation needs it); the binding raises before calling the library."""
    d, n = 4, 100
    q = si.weibull_kernel(d, n, 90, device="cuda").q
    psi = mr.psi_inverse(q)
    short = q[: n - 10].contiguous()
    cases = [
        lambda: mr.transition(psi, short),
        lambda: mr.psi_inverse_backward(psi, short),
        lambda: mr.markov_renewal_apply(psi, short[:, :, :2].contiguous()),
        lambda: mr.markov_renewal_apply_backward(psi, q[:, :, :2].contiguous(), short[:, :, :2].contiguous()),
        lambda: mr.transition_backward(psi, q, short),
        lambda: mr.transition_backward(psi, short, q),
        lambda: mr.residual_norms(q, short),
        lambda: mr.transition(q[:, :, :3].contiguous(), q),
        lambda: mr.gather_block(q, [0, 4], [1]),
        lambda: mr.scatter_block_add(torch.zeros((n, 2, 1), dtype=torch.float64, device="cuda"), d, d, [1, 1], [0]),
    ]
    for i, c in enumerate(cases):
        with pytest.raises(mr.MrinvError):
            c()
    mr.sync_status()


def test_seed_too_long_for_lds_is_reported(mr):
    """seed_m0 = 64 at d = 64 needs 70 KiB of LDS: the call returns
    MRINV_E_UNSUPPORTED instead of launching; m0 = 32 fits and matches."""
    d, n = 64, 200
    q = si.weibull_kernel(d, n, 91, device="cuda").q
    ref = mr.psi_inverse(q)
    old = mr.get_tuning()
    try:
        mr.set_tuning(seed_m0=64)
        with pytest.raises(mr.MrinvError) as ei:
            mr.psi_inverse(q)
        assert ei.value.status == 5
        mr.set_tuning(seed_m0=32)
        got = mr.psi_inverse(q)
        torch.cuda.synchronize()
        assert float((got - ref).abs().max()) <= 1e-13
    finally:
        mr.set_tuning(**old)
    mr.sync_status()
