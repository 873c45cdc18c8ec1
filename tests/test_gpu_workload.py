"""The device twin of the Chung-Lu draw writes exactly the host generator's
draws (same tables, integer arithmetic only), including failed rejections."""
import numpy as np
import pytest

import workload

pytestmark = pytest.mark.gpu


def test_device_draws_equal_host_draws():
    torch = pytest.importorskip("torch")
    for scale, first, count in ((0.001, 0, 2_000_000), (0.01, 0, 20_000_000), (0.01, 123_456_789, 1_000_003)):
        st = workload.c4_stream(scale)
        host = np.empty(count * 3, np.int32)
        k = workload._load().gsw_cl_draws(st._h, first, count, host)
        dev = torch.empty(count * 3, dtype=torch.int32, device="cuda")
        bad = st.device_draws(first, count, dev)
        d = dev.view(-1, 3).cpu().numpy()
        d = d[d[:, 0] >= 0]
        assert bad == count - k
        assert np.array_equal(d, host[:3 * k].reshape(-1, 3)), (scale, first)


def test_device_graph_equals_host_chunks():
    torch = pytest.importorskip("torch")
    st = workload.c4_stream(0.001)
    n, D, _ = workload.c4_sizes(0.001)
    dev = st.device_graph(D).cpu().numpy()
    host = np.concatenate([c.copy() for c in st.chunks(D, 300_000)])
    assert np.array_equal(dev, host)
