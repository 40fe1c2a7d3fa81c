"""The unit-rate probes behind the roofline fractions (mbkk_microbench):
every probe kind runs and reports a rate below twice its datasheet peak, and
bad arguments are rejected before any launch."""
import ctypes as C

import pytest

pytestmark = pytest.mark.gpu

# datasheet peaks per probe (lane operations or flops per second, MI355X)
PEAK = {0: 78.6e12, 1: 78.6e12, 2: 78.6e12, 3: 2.5e15, 4: 157.3e12, 5: 2.5e15}


def _probe(kind, iters, waves):
    import torch
    from paper_2410_05902_amd import _lib as L
    sink = torch.zeros(256, dtype=torch.float32, device="cuda")
    ms, ops = C.c_double(), C.c_double()
    rc = L.lib().mbkk_microbench(kind, iters, waves, C.c_void_p(torch.cuda.current_stream().cuda_stream),
                                 C.c_void_p(sink.data_ptr()), C.byref(ms), C.byref(ops))
    return rc, ms.value, ops.value


@pytest.mark.parametrize("kind", sorted(PEAK))
@pytest.mark.parametrize("waves", [1, 2])
def test_probe_runs_and_rate_is_plausible(kind, waves):
    rc, ms, ops = _probe(kind, 2000, waves)
    assert rc == 0
    assert ms > 0.0 and ops > 0.0
    rate = ops / (ms * 1e-3)
    assert 0.0 < rate < 2.0 * PEAK[kind], rate


def test_probe_rejects_bad_arguments():
    assert _probe(99, 10, 1)[0] == -1  # unknown kind
    assert _probe(0, 0, 1)[0] == -1    # no iterations
    assert _probe(0, 10, 0)[0] == -1   # waves per SIMD out of [1, 8]
    assert _probe(0, 10, 9)[0] == -1
