"""Peeling of r-hypergraphs (2 <= r <= 8) through the C ABI against the oracle, element by
element: order, round, 2-core mask, hinge position and the counts."""
import numpy as np
import pytest

import oracle
import pins

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mx():
    import torch

    import paper_1312_0526_amd as mx

    assert torch.cuda.is_available()
    mx.lib()
    return mx


@pytest.fixture(scope="module")
def o():
    return oracle.Oracle()


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def host(t, dt):
    return t.cpu().numpy().view(dt)


def _check(mx, o, edges, m, r):
    rc, ref = o.peel_r(edges, m, r)
    assert rc == 0
    got = mx.peel_r(dev(edges), m)
    assert got["n_peeled"] == ref["n_peeled"] and got["n_rounds"] == ref["n_rounds"]
    for key, dt in (("order", np.uint32), ("round", np.uint32), ("core_mask", np.uint8), ("hinge", np.uint8)):
        assert np.array_equal(host(got[key], dt), ref[key]), key
    return ref


@pytest.mark.parametrize("r", [2, 3, 4, 5, 8])
@pytest.mark.parametrize("n,gamma", [(1000, 1.5), (70_001, 1.5), (200_000, 1.2)])
def test_peel_r_matches_oracle(mx, o, r, n, gamma):
    rng = np.random.default_rng(1000 * r + n % 997)
    m = max(r, int(gamma * n))
    edges = pins.random_uniform_r(n, m, r, rng)
    if n == 1000:
        edges = np.concatenate([edges, edges[:50]])  # duplicates end in the 2-core
    _check(mx, o, edges, m, r)


def test_peel_r4_threshold_sides(mx, o):
    # r = 4 peels completely above gamma* = 1.295 vertices per edge; below it the core holds
    # the closed-form fraction of the edges
    rng = np.random.default_rng(4)
    n = 300_000
    full = _check(mx, o, pins.random_uniform_r(n, int(1.40 * n), 4, rng), int(1.40 * n), 4)
    assert full["n_peeled"] == n
    part = _check(mx, o, pins.random_uniform_r(n, int(1.20 * n), 4, rng), int(1.20 * n), 4)
    assert abs(1 - part["n_peeled"] / n - pins.core_fraction_closed_form(1.20, 4)) < 0.01


def test_peel_r_long_chain(mx, o):
    n = 2001
    edges = np.array([[i, i + 1, i + 2, i + 3] for i in range(n)], np.uint32)
    ref = _check(mx, o, edges, n + 3, 4)
    assert ref["n_rounds"] > 900


def test_peel_r3_equals_peel(mx, o):
    rng = np.random.default_rng(33)
    edges = pins.random_uniform_r(50_000, 60_000, 3, rng)
    a, b = mx.peel(dev(edges), 60_000), mx.peel_r(dev(edges), 60_000)
    for key, dt in (("order", np.uint32), ("round", np.uint32), ("core_mask", np.uint8), ("hinge", np.uint8)):
        assert np.array_equal(host(a[key], dt), host(b[key], dt)), key


def test_peel_r_empty_and_errors(mx):
    import ctypes as C

    import torch

    got = mx.peel_r(dev(np.zeros((0, 4), np.uint32)), 10)
    assert got["n_peeled"] == 0 and got["n_rounds"] == 0
    with pytest.raises(mx.MphxError) as ei:
        mx.peel_r(dev(np.array([[0, 1, 1, 2]], np.uint32)), 5)
    assert ei.value.status == mx.EINVAL
    with pytest.raises(mx.MphxError) as ei:
        mx.peel_r(dev(np.array([[0, 7]], np.uint32)), 5)
    assert ei.value.status == mx.EINVAL
    star = np.array([[0, 1 + i] for i in range(256)], np.uint32)
    with pytest.raises(mx.MphxError) as ei:
        mx.peel_r(dev(star), 300)
    assert ei.value.status == mx.ERANGE
    assert mx.peel_r(dev(star[:255]), 300)["n_peeled"] == 255
    # r outside [2, 8] is refused before any device work
    edges = dev(np.arange(9, dtype=np.uint32).reshape(1, 9))
    out = [torch.empty(1, dtype=torch.int32, device="cuda") for _ in range(2)]
    mask = torch.empty(1, dtype=torch.uint8, device="cuda")
    ws = torch.empty(1 << 16, dtype=torch.uint8, device="cuda")
    rc = mx.lib().mphx_peel_r(edges.data_ptr(), 1, 9, 9, out[0].data_ptr(), out[1].data_ptr(), mask.data_ptr(),
                              None, ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream, None)
    assert rc == mx.EINVAL
    assert mx.lib().mphx_peel_r_workspace_bytes(10, 20, 9) == 0
