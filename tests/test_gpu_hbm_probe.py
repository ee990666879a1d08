"""The HBM probe (mrinv_hbm_probe), the measured ceiling that bench.py reports
beside the published 8 TB/s: each pattern must touch exactly the elements it
claims, once per launch, or its rate would mean nothing."""
import pytest
import torch

pytestmark = pytest.mark.gpu

MIB = 1 << 20


@pytest.fixture(scope="module")
def mr():
    import paper_2605_30379_amd as m
    assert torch.cuda.is_available()
    m.lib()
    return m


def test_copy_pattern_copies_the_first_half(mr):
    g = torch.Generator(device="cuda").manual_seed(11)
    buf = torch.rand(8 * MIB // 8, dtype=torch.float64, device="cuda", generator=g)
    first = buf[: buf.numel() // 2].clone()
    rate = mr.hbm_probe(buf, "copy", reps=2)
    torch.cuda.synchronize()
    assert rate > 0
    assert torch.equal(buf[buf.numel() // 2:], first)
    assert torch.equal(buf[: buf.numel() // 2], first)


@pytest.mark.parametrize("pattern", ["pass_first", "pass_last"])
@pytest.mark.parametrize("lanes", [8, 16, 32])
def test_pass_patterns_visit_every_element_once_per_launch(mr, pattern, lanes):
    # 48 MiB: the largest power-of-two row count that fits is 1024 rows of
    # 2048 complex doubles (32 MiB); the tail must stay untouched.
    z = torch.zeros(48 * MIB // 8, dtype=torch.float64, device="cuda")
    z[1::2] = 7.0                      # imaginary parts
    tail = 32 * MIB // 8
    z[tail:] = -3.0
    rate = mr.hbm_probe(z, pattern, lanes=lanes, reps=3)
    torch.cuda.synchronize()
    assert rate > 0
    head = z[:tail].view(-1, 2)
    assert torch.all(head[:, 0] == 3.0)
    assert torch.all(head[:, 1] == 7.0)
    assert torch.all(z[tail:] == -3.0)


def test_probe_arguments_are_checked_before_any_launch(mr):
    small = torch.zeros(16 * MIB // 8, dtype=torch.float64, device="cuda")
    for kw in (dict(pattern="pass_first", lanes=16), dict(pattern="pass_last", lanes=12)):
        with pytest.raises(mr.MrinvError):
            mr.hbm_probe(small, **kw)
    with pytest.raises(mr.MrinvError):
        mr.hbm_probe(torch.zeros(MIB // 8, dtype=torch.float64, device="cuda"), "copy")
    with pytest.raises(mr.MrinvError):
        mr.hbm_probe(small, "copy", reps=0)
    torch.cuda.synchronize()
    assert torch.all(small == 0)
