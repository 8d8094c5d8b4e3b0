"""Proposer kernels (features, FP32 MLP forward / gradient / Adam, top-k,
rank labels) against numpy references.

The MLP is FP32 on both the device and in these checks' error bounds: a
sum of k products rounded in FP32 is within about k * 2^-24 of the exact
sum of the absolute products, so each check computes that absolute-value
bound in float64 and allows a multiple of it.  Top-k ids and rank labels
are exact (integer decisions taken on the same keys)."""
import numpy as np
import pytest
import torch

from homln_inputs import configs as C
from oracle import oracle as O
from tests.gpu_common import csr_np, graph_dev, say

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2207_11662_amd")

F, H = 12, 64
U = 2.0 ** -24


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + F * H].reshape(F, H); o += F * H
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def forward_ref(p, X):
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ W1 + b1
    h1 = np.maximum(a1, 0)
    a2 = h1 @ W2 + b2
    h2 = np.maximum(a2, 0)
    y = h2 @ w3 + b3
    # magnitudes the rounding errors scale with
    A1 = np.abs(X) @ np.abs(W1) + np.abs(b1)
    A2 = np.maximum(A1, 0) @ np.abs(W2) + np.abs(b2)
    Y = A2 @ np.abs(w3) + abs(b3)
    return dict(a1=a1, h1=h1, a2=a2, h2=h2, y=y, A1=A1, A2=A2, Y=Y)


def y_err(f):
    """Bound on the FP32 forward's error in y."""
    return 2 * (F + 2 * H + 4) * U * f["Y"]


def grad_ref(p, X, t):
    """Gradient of mean((y - t)^2) and an absolute-value bound per entry."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    f = forward_ref(p, X)
    n = X.shape[0]
    X = np.asarray(X, dtype=np.float64)
    r = f["y"] - t
    dy = 2.0 * r / n
    m2 = (f["a2"] > 0).astype(np.float64)
    m1 = (f["a1"] > 0).astype(np.float64)
    d2 = dy[:, None] * w3[None, :] * m2
    d1 = (d2 @ W2.T) * m1
    g = np.concatenate([(X.T @ d1).ravel(), d1.sum(0), (f["h1"].T @ d2).ravel(), d2.sum(0),
                        f["h2"].T @ dy, [dy.sum()]])
    Dy = np.abs(dy) + 2.0 * y_err(f) / n                 # dy plus the error y carries
    D2 = Dy[:, None] * np.abs(w3)[None, :] * m2
    D1 = (D2 @ np.abs(W2).T) * m1
    G = np.concatenate([(np.abs(X).T @ D1).ravel(), D1.sum(0), (f["A2"].T @ D2).ravel(), D2.sum(0),
                        f["A2"].T @ Dy, [Dy.sum()]])
    loss = float(np.mean(r * r))
    return g, G, loss, f


def away_from_kinks(p, X, frac=1e-4):
    """Rows whose every pre-activation is clear of 0 by frac of its bound, so
    that FP32 and FP64 take the same ReLU branches."""
    f = forward_ref(p, X)
    ok = np.all(np.abs(f["a1"]) > frac * f["A1"], axis=1) & np.all(np.abs(f["a2"]) > frac * f["A2"], axis=1)
    return X[ok]


def new_params(seed):
    npar = P.mlp_param_count()
    assert npar == F * H + H + H * H + H + H + 1
    p = torch.empty(npar, dtype=torch.float32, device="cuda")
    m = torch.full_like(p, 7.0)
    v = torch.full_like(p, 7.0)
    P.hln_mlp_init(p, m, v, seed=seed)
    torch.cuda.synchronize()
    assert float(m.abs().max()) == 0 and float(v.abs().max()) == 0
    return p, m, v


def test_init_glorot_ranges_and_zero_biases():
    p, _, _ = new_params(3)
    W1, b1, W2, b2, w3, b3 = unpack(p.cpu().numpy())
    for W, fan in ((W1, F + H), (W2, 2 * H), (w3, H + 1)):
        lim = np.sqrt(6.0 / fan)
        assert np.abs(W).max() <= lim and np.abs(W).max() > 0.9 * lim
        assert abs(W.mean()) < 4 * lim / np.sqrt(3 * W.size)      # 4 sigma of a uniform mean
    assert not b1.any() and not b2.any() and b3 == 0
    q, _, _ = new_params(3)
    r, _, _ = new_params(4)
    assert torch.equal(p, q) and not torch.equal(p, r)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 40001])
def test_forward_matches_fp64(n):
    rng = np.random.default_rng(n)
    p, _, _ = new_params(11)
    # non-zero biases so that every parameter group matters
    pn = p.cpu().numpy()
    pn[F * H:F * H + H] = rng.normal(0, 0.1, H)
    pn[F * H + H + H * H:F * H + 2 * H + H * H] = rng.normal(0, 0.1, H)
    pn[-1] = 0.3
    p = torch.from_numpy(pn).cuda()
    X = rng.normal(0, 1, (n, F)).astype(np.float32)
    y = P.hln_mlp_forward(p, torch.from_numpy(X).cuda())
    torch.cuda.synchronize()
    f = forward_ref(pn, X)
    err = np.abs(y.cpu().numpy() - f["y"])
    bound = y_err(f) + 1e-30
    say("forward n", n, "max err/bound", float((err / bound).max()))
    assert np.all(err <= bound)


def test_gradient_loss_and_adam_step():
    rng = np.random.default_rng(5)
    p, m, v = new_params(21)
    pn = p.cpu().numpy()
    X = away_from_kinks(pn, rng.normal(0, 1, (6000, F)).astype(np.float32))
    n = X.shape[0]
    say("rows clear of ReLU kinks", n)
    t = rng.uniform(0, 1, n).astype(np.float32)
    Xd, td = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    # lr = 0: parameters stay, the first moment is (1 - beta1) * gradient
    P.hln_mlp_train_step(p, m, v, 1, 0.0, Xd, td, loss=loss)
    torch.cuda.synchronize()
    assert torch.equal(p.cpu(), torch.from_numpy(pn))
    g_dev = m.cpu().numpy().astype(np.float64) / np.float64(np.float32(1.0) - np.float32(0.9))   # m = (1 - beta1) g
    g, G, loss_ref, f = grad_ref(pn, X, t)
    bound = (4 * (3 * H + F + n // 64 + 64) * U) * G + 1e-30
    err = np.abs(g_dev - g)
    say("grad max err/bound", float((err / bound).max()))
    assert np.all(err <= bound)
    c1 = np.float64(np.float32(1.0) - np.float32(0.9))      # 1 - beta1 and 1 - beta2 as the device rounds them
    c2 = np.float64(np.float32(1.0) - np.float32(0.999))
    vv = v.cpu().numpy().astype(np.float64)
    assert np.allclose(vv, c2 * g_dev ** 2, rtol=1e-5, atol=0)
    # loss: FP32 error of y propagated through r^2, plus the summation
    r = f["y"] - t
    ey = y_err(f)
    lbound = np.mean(2 * np.abs(r) * ey + ey * ey) + 2 * (64 + n // 64) * U * np.mean(r * r + 2 * np.abs(r) * ey)
    say("loss", float(loss.item()), loss_ref, lbound)
    assert abs(float(loss.item()) - loss_ref) <= lbound
    # Adam step 1 from zero moments, checked from the device's own moments
    p2, m2, v2 = new_params(21)
    lr = 1e-2
    P.hln_mlp_train_step(p2, m2, v2, 1, lr, Xd, td)
    torch.cuda.synchronize()
    mm = m2.cpu().numpy().astype(np.float64)
    vv = v2.cpu().numpy().astype(np.float64)
    assert np.array_equal(m2.cpu().numpy(), m.cpu().numpy())       # deterministic
    exp = pn - np.float64(np.float32(lr)) * (mm / c1) / (np.sqrt(vv / c2) + 1e-8)
    got = p2.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - exp) <= 1e-5 * lr + 4 * np.abs(exp) * U)


def test_training_is_deterministic_and_fits():
    rng = np.random.default_rng(9)
    n = 20000
    X = rng.normal(0, 1, (n, F)).astype(np.float32)
    t = (1 / (1 + np.exp(-(X[:, 0] - 0.5 * X[:, 3] + 0.3 * X[:, 7] * X[:, 2])))).astype(np.float32)
    Xd, td = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    runs = []
    for rep in range(2):
        p, m, v = new_params(1)
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        ws = None
        hist = []
        for step in range(1, 301):
            ws = P.hln_mlp_train_step(p, m, v, step, 3e-3, Xd, td, loss=loss, ws=ws)
            if step in (1, 300):
                torch.cuda.synchronize()
                hist.append(float(loss.item()))
        torch.cuda.synchronize()
        runs.append((p.cpu().clone(), hist))
    say("loss first/last", runs[0][1])
    assert torch.equal(runs[0][0], runs[1][0]) and runs[0][1] == runs[1][1]
    assert runs[0][1][1] < 0.1 * runs[0][1][0]


def log_rank(s):
    """log((n+1)/(g+1)) / log(n+1), g = number of strictly larger scores."""
    n = len(s)
    asc = np.sort(np.asarray(s, dtype=np.float64))
    g = n - np.searchsorted(asc, np.asarray(s, dtype=np.float64), side="right")
    return (np.log((n + 1.0) / (g + 1.0)) / np.log(n + 1.0)).astype(np.float32)


def ref_order(s):
    return np.lexsort((np.arange(len(s)), -np.asarray(s, dtype=np.float64)))


@pytest.mark.parametrize("n,dtype,ties", [(1, torch.float64, False), (7, torch.float32, True),
                                          (1000, torch.float64, True), (1000, torch.float32, False),
                                          (100003, torch.float64, True), (100003, torch.float32, True)])
def test_topk_and_rank_labels(n, dtype, ties):
    rng = np.random.default_rng(n)
    s = rng.normal(0, 1, n)
    if ties:
        s = np.round(s * 4) / 4                        # many equal scores, +0.0 and -0.0 among them
        s[rng.random(n) < 0.05] = -0.0
    s = s.astype(np.float64 if dtype == torch.float64 else np.float32)
    sd = torch.from_numpy(s).cuda()
    order = ref_order(s)
    for k in sorted({0, 1, 2, n // 2, n}):
        if k > n:
            continue
        ids = P.hln_topk(sd, k)
        torch.cuda.synchronize()
        assert np.array_equal(ids.cpu().numpy(), order[:k]), (n, k)
        ids_set = P.hln_topk(sd, k, as_set=True)          # the same set, ascending ids
        torch.cuda.synchronize()
        assert np.array_equal(ids_set.cpu().numpy(), np.sort(order[:k])), (n, k)
    lab = P.hln_rank_labels(sd)
    torch.cuda.synchronize()
    exp = log_rank(s)
    # double logarithms may differ in the last bit, which can move the float
    # rounding by one unit
    got = lab.cpu().numpy()
    assert np.all(np.abs(got.view(np.int32) - exp.view(np.int32)) <= 1)
    # non-increasing along the score order
    assert np.all(np.diff(got[order].astype(np.float64)) <= 0)


def test_features_match_fp64():
    h = C.config1()
    n = h.n
    layers = [csr_np(n, *e) for e in h.layers]
    graphs, Ss, Rs, h2s, ref = [], [], [], [], []
    for rp, ci in layers:
        S, R, H2, _, _ = O.bfs_sums(rp, ci, extras=True)
        cc = O.closeness_wf(n, S, R)
        graphs.append(graph_dev(P, rp, ci))
        Ss.append(torch.from_numpy(S).cuda())
        Rs.append(torch.from_numpy(R).cuda())
        h2s.append(torch.from_numpy(H2.astype(np.int32)).cuda())
        md = len(ci) / n
        ref.append(np.stack([np.log1p(np.diff(rp) / md), cc, np.log1p(H2 / md ** 2)], 1))
    X = P.hln_proposer_features(graphs, Ss, Rs, h2s)
    torch.cuda.synchronize()
    V = np.stack(ref, 0)                                   # [r, n, 3]
    exp = np.stack([V.min(0), V.max(0), V.mean(0), V.std(0)], 2).reshape(n, F)
    got = X.cpu().numpy().astype(np.float64)
    scale = np.abs(V).max(0).repeat(4, axis=1).reshape(n, F) + 1e-30
    err = np.abs(got - exp)
    say("features max err/scale", float((err / scale).max()))
    assert np.all(err <= 16 * U * scale + 1e-7)
    # a vertex isolated in every layer: zero closeness
    iso = np.flatnonzero(np.all([np.diff(rp) == 0 for rp, _ in layers], axis=0))
    for u in iso:
        assert got[u, 4:8].tolist() == [0, 0, 0, 0]
