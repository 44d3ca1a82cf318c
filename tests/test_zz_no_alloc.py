"""GPU check of osm_net_loss_grad_noalloc, the entry point that allocates
nothing: through the C ABI, on two calls in a row (the second with fewer
and shorter traces, so stale partials of the first would show), its loss
and gradient must equal those of osm_net_loss_grad bit for bit (same
kernels, same order of summation), and sizes beyond its static workspace
must be rejected before anything is enqueued."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import nn  # noqa: E402
from workloads import net_init  # noqa: E402

DEV = "cuda:0"


def _data(T, L, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((T, nn.CIN, L)).astype(np.float32)
    t = (0.3 * rng.standard_normal((T, nn.COUT, L))).astype(np.float32)
    return torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV)


def test_noalloc_loss_grad_matches_the_allocating_entry_point():
    from paper_1603_05110_amd import osm
    net = osm.OsmNet(64, DEV)
    net.set_params(torch.from_numpy(net_init(3) * 2.0))
    grad = torch.empty(osm.NET_NPARAMS, dtype=torch.float32, device=DEV)
    loss = torch.empty(1, dtype=torch.float64, device=DEV)
    for T, L, seed in [(37, 1025, 11), (5, 150, 12)]:
        print(f"noalloc loss/grad T={T} L={L}", flush=True)
        sys.stdout.flush()
        x, t = _data(T, L, seed)
        grad.fill_(float("nan"))
        loss.fill_(float("nan"))
        net.loss_grad_noalloc(x, t, grad, loss)
        torch.cuda.synchronize()
        ref_loss, ref_grad = net.loss_grad(x, t)
        got = grad.cpu().numpy()
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, ref_grad.cpu().numpy())
        assert loss.item() == ref_loss
        # the same call without a loss pointer writes the gradient alike
        grad.fill_(0.0)
        net.loss_grad_noalloc(x, t, grad)
        torch.cuda.synchronize()
        assert np.array_equal(grad.cpu().numpy(), ref_grad.cpu().numpy())

    # beyond the static workspace: rejected, nothing written
    T = osm.NET_NOALLOC_MAX_TRACES + 1
    x, t = _data(T, 8, 13)
    grad.fill_(7.0)
    with pytest.raises(osm.OsmError) as e:
        net.loss_grad_noalloc(x, t, grad, loss)
    assert e.value.status == osm.OSM_EINVAL
    assert "OSM_NET_NOALLOC_MAX_TRACES" in str(e.value)
    torch.cuda.synchronize()
    assert bool(torch.all(grad == 7.0))
    # the largest size it accepts
    x, t = _data(osm.NET_NOALLOC_MAX_TRACES, 70, 14)
    net.loss_grad_noalloc(x, t, grad, loss)
    torch.cuda.synchronize()
    ref_loss, ref_grad = _reference_with_room(osm, net, x, t)
    assert np.array_equal(grad.cpu().numpy(), ref_grad)
    assert loss.item() == ref_loss
    net.close()


def _reference_with_room(osm, net, x, t):
    """osm_net_loss_grad of a network whose workspace holds all T traces."""
    big = osm.OsmNet(x.shape[0], DEV)
    big.set_params(net.get_params())
    l, g = big.loss_grad(x, t)
    out = g.cpu().numpy()
    big.close()
    return l, out
