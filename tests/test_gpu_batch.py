"""GPU: many points per call (grouped by lattice size, batched launches),
bitwise independence of a point's result from its batch, batched gradients,
and replay of a captured HIP graph of a whole call."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1412_8754_amd import OMEGA_FP32_COMP, OMEGA_FP64, api  # noqa: E402
from paper_1412_8754_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
M = W.DEFAULT_MODEL


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def mixed_points(n, seed):
    rng = np.random.default_rng(seed)
    sizes = [(16, 16), (24, 10), (9, 33), (32, 32)]
    pts = []
    for i in range(n):
        Lx, Ly = sizes[int(rng.integers(0, len(sizes)))]
        pts.append((float(rng.uniform(-0.3, 0.3)), float(rng.choice([0.0, 0.003, 0.04])), Lx, Ly))
    return pts


@pytest.mark.parametrize("prec", [OMEGA_FP64, OMEGA_FP32_COMP])
def test_batch_is_bitwise_equal_to_single_point_calls(prec):
    pts = mixed_points(9, 5)
    delta = np.linspace(0, 0.6, 40)
    q = np.array([[0.0, 0.0], [0.25, 0.0], [0.1, 0.2]])
    say(f"batch of {len(pts)} mixed points, prec {prec}")
    idx, omin, rows, om = api.argmin(M, pts, delta, q, 3, prec)
    torch.cuda.synchronize()
    om = om.cpu().numpy()
    for i, pt in enumerate(pts):
        _, _, _, om1 = api.argmin(M, [pt], delta, q, 3, prec)
        torch.cuda.synchronize()
        assert np.array_equal(om[i].view(np.uint64), om1.cpu().numpy()[0].view(np.uint64)), i


def test_many_points_beyond_one_fill_launch():
    pts = mixed_points(300, 6)
    delta = np.linspace(0, 0.6, 16)
    q = W.q_axis(4, np.pi / 64)
    say(f"batch of {len(pts)} points")
    idx, omin, rows, om = api.argmin(M, pts, delta, q, 3)
    torch.cuda.synchronize()
    om = om.cpu().numpy()
    sel = [0, 1, 127, 128, 129, 255, 256, 299]
    ref = oracle.omega_grid(M, [pts[i] for i in sel], delta, q, 3)
    N = np.array([pts[i][2] * pts[i][3] for i in sel]).reshape(-1, 1, 1, 1)
    err = np.abs(om[sel] - ref)
    assert (err <= 1e-12 * np.abs(ref) + 1e-13 * N).all(), np.max(err / np.abs(ref))
    _, ridx, _, _ = oracle.omega_argmin(M, [pts[i] for i in sel], delta, q, 3)
    np.testing.assert_array_equal(idx.cpu().numpy()[sel], ridx)


def test_one_point_per_batch_reuses_the_workspace_queues():
    """16384 Q x 2 bands = 32768 rows allow one point per batch (the grid's
    z extent is 65535), so these 5 points run as 5 batches, one after the
    other, through the same workspace and the same work-queue counters."""
    rng = np.random.default_rng(11)
    pts = [(float(rng.uniform(-0.2, 0.2)), float(rng.choice([0.0, 0.004, 0.05])), L, L)
           for L in (8, 6, 8, 4, 8)]
    delta = np.array([0.0, 0.15, 0.4])
    q = rng.uniform(-np.pi, np.pi, size=(16384, 2))
    q[:64, 1] = 0.0
    q[:16, 0] = 2 * np.pi * np.arange(16) / 8     # some lattice momenta too
    say(f"{len(pts)} points x {len(q)} Q, one point per batch")
    idx, omin, rows, om = api.argmin(M, pts, delta, q, 3)
    torch.cuda.synchronize()
    om = om.cpu().numpy()
    ref = oracle.omega_grid(M, pts, delta, q, 3)
    N = np.array([p[2] * p[3] for p in pts]).reshape(-1, 1, 1, 1)
    err = np.abs(om - ref)
    assert (err <= 1e-12 * np.abs(ref) + 1e-13 * N).all(), np.max(err / np.abs(ref))
    _, ridx, _, _ = oracle.omega_argmin(M, pts, delta, q, 3)
    np.testing.assert_array_equal(idx.cpu().numpy(), ridx)


def test_batched_gradients_against_oracle():
    pts = mixed_points(200, 7)
    rng = np.random.default_rng(8)
    delta = rng.uniform(0, 0.6, size=(len(pts), 2))
    q = rng.uniform(-0.4, 0.4, size=(len(pts), 2, 2))
    say(f"batched gradient over {len(pts)} points")
    om, gd, gq, gm = (t.cpu().numpy() for t in api.grad(M, pts, delta, q, 3))
    sel = [0, 3, 127, 128, 199]
    for b in range(2):
        rom, rgd, rgq, rgm = oracle.omega_grad(M, [pts[i] for i in sel], delta[sel, b],
                                               q[sel, b], b)
        N = np.array([pts[i][2] * pts[i][3] for i in sel], dtype=float)
        for got, ref in ((om[sel, b], rom), (gd[sel, b], rgd), (gq[sel, b, 0], rgq[:, 0]),
                         (gq[sel, b, 1], rgq[:, 1]), (gm[sel, b], rgm)):
            assert (np.abs(got - ref) <= 1e-12 * np.abs(ref) + 1e-13 * N).all(), (got, ref)


def test_call_on_a_side_stream_matches_the_current_stream():
    """A call given another stream waits for the current stream's work (its
    inputs, outputs and workspace are made there) and returns what the same
    call on the current stream returns, bitwise, for device and host inputs."""
    pts = mixed_points(4, 11)
    delta = torch.linspace(0, 0.6, 33, dtype=torch.float64, device="cuda")
    q = torch.tensor([[0.0, 0.0], [0.2, 0.0]], dtype=torch.float64, device="cuda")
    say("case: argmin on a side stream, 4 points, 33 Delta, 2 Q")
    ref = api.argmin(M, pts, delta, q, 3, OMEGA_FP64)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    for dl, qq in ((delta, q), (delta.cpu().numpy(), q.cpu().numpy())):
        got = api.argmin(M, pts, dl, qq, 3, OMEGA_FP64, stream=s)
        s.synchronize()
        for a, b in zip(got, ref):
            assert torch.equal(a, b)


def test_captured_graph_replays_match_eager():
    pts = mixed_points(5, 9)
    dev = "cuda"
    delta = torch.linspace(0, 0.6, 48, dtype=torch.float64, device=dev)
    q = torch.tensor([[0.0, 0.0], [0.3, 0.0]], dtype=torch.float64, device=dev)
    nb, nq, nd = 2, q.shape[0], delta.numel()
    ws = torch.empty(api.workspace_bytes(pts, nd, nq, 3, OMEGA_FP64), dtype=torch.uint8,
                     device=dev)
    say("graph capture of omega_argmin")
    # eager reference
    idx0, omin0, rows0, om0 = api.argmin(M, pts, delta, q, 3, workspace=ws)
    torch.cuda.synchronize()
    om0 = om0.clone()
    idx0 = idx0.clone()
    # capture (outputs allocated inside the graph's private pool)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        api.argmin(M, pts, delta, q, 3, workspace=ws)   # warm-up on the side stream
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            idx_g, omin_g, rows_g, om_g = api.argmin(M, pts, delta, q, 3, workspace=ws)
    torch.cuda.synchronize()
    for rep in range(3):
        om_g.fill_(float("nan"))
        idx_g.fill_(-7)
        # unrelated eager work between replays
        junk = torch.randn(1 << 16, dtype=torch.float64, device=dev).sum()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(om_g.cpu().numpy().view(np.uint64), om0.cpu().numpy().view(np.uint64)), rep
        assert torch.equal(idx_g, idx0), rep
        assert bool(torch.isfinite(junk))


def test_phase_diagram_fp32c_minima_match_fp64():
    """16 x 16 (h, T) points at L = 256 (h up to 0.4, T up to 0.05): the
    FP32-compensated search returns the FP64 global minimum at every point
    and band (its candidates within the FP32 error band are re-evaluated in
    FP64 before the tie rule picks one)."""
    cfg = W.phase_config(16, 16, fixed_L=256)
    pts, delta, q = cfg["pts"], cfg["delta"], cfg["q"]
    say(f"phase diagram {len(pts)} points at L=256, FP64 vs FP32c")
    idx64, omin64, _, om64 = api.argmin(M, pts, delta, q, 3, OMEGA_FP64)
    idx32, omin32, _, om32 = api.argmin(M, pts, delta, q, 3, OMEGA_FP32_COMP)
    torch.cuda.synchronize()
    idx64, idx32 = idx64.cpu().numpy(), idx32.cpu().numpy()
    om64, om32 = om64.cpu().numpy(), om32.cpu().numpy()
    rel = np.max(np.abs(om32 - om64) / np.abs(om64))
    diff = np.argwhere((idx64 != idx32).any(axis=-1))
    say(f"max rel {rel:.2e}; {len(diff)} of {idx64.shape[0] * 2} minima differ")
    assert rel <= 1e-7
    assert len(diff) == 0, diff.tolist()
    np.testing.assert_allclose(omin32.cpu().numpy(), omin64.cpu().numpy(), rtol=1e-12, atol=0)
