"""Surrogate network on the GPU (BF16 matrix-core products, FP32 accumulation),
through the C-ABI of include/alelb_mlp.h, against the FP64 oracle
oracle/mlp_oracle.py, and the trained surrogate against the solver.

Tolerances.
- Products of small integers are exact in BF16 and in FP32 sums of up to 256
  terms, so the GEMM must reproduce integer matrix products bit for bit
  (this pins the matrix-core operand and result layout).
- Against the oracle that rounds every product's operands to BF16 as the GPU
  does, forward outputs and gradients differ only by FP32 accumulation and
  FP32 activations, and by the rare operand whose BF16 rounding flips with the
  last FP32 bit.  A flip changes one product by at most one BF16 ulp (2^-8
  relative), so element by element no entry of a tensor may differ by more
  than 2^-8 of that tensor's largest oracle magnitude; over the whole tensor
  the relative L2 error stays below 1e-3.
- Adam, step after step, against the oracle's update fed the GPU's own
  gradients: the FP32 parameters may differ from the FP64 ones by the FP32
  rounding of a dozen updates, far below 1e-3 of the learning rate.
- Against the plain FP64 oracle the BF16 operands give about 1% (reported).
"""

import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

WIDTHS = [5, 256, 256, 256, 256]


@pytest.fixture(scope="module")
def mlp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2002_04353_amd import mlp as Mm
    Mm.load()
    return Mm


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


ELEM_TOL = 2.0 ** -8  # one BF16 ulp of the tensor's scale


def _elem(a, b):
    """Largest element-wise difference over the tensor's largest magnitude."""
    a, b = np.ravel(np.asarray(a, np.float64)), np.ravel(np.asarray(b, np.float64))
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("M,N,K", [(70, 45, 100), (64, 256, 256), (1, 1, 1), (33, 17, 5), (300, 256, 32),
                                   (16384, 256, 256), (20001, 300, 96)])
def test_gemm_reproduces_integer_products(mlp, M, N, K):
    import torch
    rng = np.random.default_rng(M * 1000 + N)
    A = rng.integers(-8, 9, size=(M, K))
    B = rng.integers(-8, 9, size=(K, N))
    ta = torch.tensor(A, dtype=torch.bfloat16, device="cuda").contiguous()
    tb = torch.tensor(B, dtype=torch.bfloat16, device="cuda").contiguous()
    tc = torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")
    mlp.gemm_bf16(ta.data_ptr(), tb.data_ptr(), tc.data_ptr(), M, N, K)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(tc.cpu().numpy(), (A @ B).astype(np.float32))


def _net(mlp, oracle_params, batch):
    net = mlp.MLP(WIDTHS, batch, stream=0)
    net.set_params(oracle_params.astype(np.float32))
    return net


def _problem(seed=0, batch=300):
    from oracle import mlp_oracle as O
    rng = np.random.default_rng(seed)
    p = O.init_params(WIDTHS, seed=seed)
    # non-zero biases, exactly representable in FP32
    p = p.astype(np.float32).astype(np.float64)
    for l, (W, b) in enumerate(O.unpack(p, WIDTHS)):
        b[:] = rng.uniform(-0.2, 0.2, b.size).astype(np.float32)
    X = rng.uniform(-1, 1, (batch, WIDTHS[0])).astype(np.float32)
    T = rng.uniform(-1, 1, (batch, WIDTHS[-1])).astype(np.float32)
    return O, p, X, T


def test_forward_matches_oracle(mlp):
    O, p, X, T = _problem(0)
    net = _net(mlp, p, X.shape[0])
    y = net.forward(X)
    y16, _ = O.forward(p, WIDTHS, X.astype(np.float64), bf16=True)
    y64, _ = O.forward(p, WIDTHS, X.astype(np.float64))
    e16, e64, x16 = _rel(y, y16), _rel(y, y64), _elem(y, y16)
    print(f"forward: rel L2 vs BF16-operand oracle {e16:.2e} (element-wise {x16:.2e}), vs FP64 oracle {e64:.2e}",
          flush=True)
    assert e16 < 1e-3 and x16 < ELEM_TOL
    assert e64 < 3e-2
    net.close()


@pytest.mark.parametrize("batch", [300, 4133])
def test_gradients_match_oracle(mlp, batch):
    # 4133 rows: the weight gradients split K = batch into 7 chunks (the last
    # one ragged), and the bias gradients add 65 row chunks' column sums
    O, p, X, T = _problem(1, batch=batch)
    net = _net(mlp, p, X.shape[0])
    loss, g = net.gradients(X, T)
    l16, g16 = O.loss_and_grad(p, WIDTHS, X.astype(np.float64), T.astype(np.float64), bf16=True)
    assert abs(loss - l16) < 1e-4 * l16
    for l, ((gw, gb), (ow, ob)) in enumerate(zip(O.unpack(g.astype(np.float64), WIDTHS), O.unpack(g16, WIDTHS))):
        ew, eb = _rel(gw, ow), _rel(gb, ob)
        xw, xb = _elem(gw, ow), _elem(gb, ob)
        print(f"layer {l}: rel L2 of dW {ew:.2e}, of db {eb:.2e}; element-wise {xw:.2e}, {xb:.2e}", flush=True)
        assert ew < 1e-3 and eb < 1e-3, l
        assert xw < ELEM_TOL and xb < ELEM_TOL, l
    net.close()


def test_train_steps_match_single_steps(mlp):
    """ale_mlp_train_steps does what the same number of ale_mlp_train_step calls
    do, bit for bit: every loss and every final parameter, across the
    1024-step boundary where losses are copied back, and on later runs with
    another batch size and other Adam constants.  Bad arguments are rejected
    and leave the parameters alone."""
    from paper_2002_04353_amd import alelb
    O, p, X, T = _problem(3, batch=64)
    n = 1030
    lrs = (1e-3 * (1.0 + np.cos(np.pi * np.arange(n) / n)) / 2 + 1e-5).astype(np.float32)
    a, b = _net(mlp, p, X.shape[0]), _net(mlp, p, X.shape[0])
    la = a.train_steps(X, T, lrs)
    lb = np.array([b.train_step(X, T, lr=float(lr)) for lr in lrs])
    np.testing.assert_array_equal(la, lb)
    np.testing.assert_array_equal(a.params(), b.params())
    assert lb[-1] < 0.5 * lb[0]
    for rows, b1, b2 in ((40, 0.8, 0.99), (64, 0.9, 0.999)):
        la = a.train_steps(X[:rows], T[:rows], lrs[:25], beta1=b1, beta2=b2)
        lb = np.array([b.train_step(X[:rows], T[:rows], lr=float(lr), beta1=b1, beta2=b2) for lr in lrs[:25]])
        np.testing.assert_array_equal(la, lb)
        np.testing.assert_array_equal(a.params(), b.params())
    before = a.params()
    for bad in ([], [1e-3, -1.0]):
        with pytest.raises(alelb.AleLbError) as e:
            a.train_steps(X, T, bad)
        assert e.value.code == alelb.EINVAL
    np.testing.assert_array_equal(a.params(), before)
    a.close()
    b.close()


def test_first_adam_step_matches_oracle(mlp):
    O, p, X, T = _problem(2)
    net = _net(mlp, p, X.shape[0])
    lr = 1e-3
    net.train_step(X, T, lr=lr)
    p1 = net.params().astype(np.float64)
    _, g = O.loss_and_grad(p, WIDTHS, X.astype(np.float64), T.astype(np.float64), bf16=True)
    q1, _, _ = O.adam_step(p, g, np.zeros_like(p), np.zeros_like(p), 1, lr)
    sel = np.abs(g) > 1e-3 * np.max(np.abs(g))  # away from g ~ 0, where the first step's sign is fragile
    assert sel.mean() > 0.5
    assert np.max(np.abs(p1[sel] - q1[sel])) < 2e-3 * lr
    net.close()


def test_adam_steps_match_oracle(mlp):
    """Adam step after step, with its bias corrections, each compared with the
    oracle's update (oracle/mlp_oracle.adam_step, FP64) fed the gradient the
    GPU computes at its current parameters: twelve steps with one set of
    constants, then, after ale_mlp_set_params (which restarts the moments and
    the step count), four with another."""
    O, p, X, T = _problem(4, batch=128)
    net = _net(mlp, p, X.shape[0])
    worst, moved = 0.0, 0.0
    for n, (lr, b1, b2) in ((12, (1e-3, 0.9, 0.999)), (4, (5e-4, 0.8, 0.99))):
        q = net.params().astype(np.float64)
        net.set_params(q.astype(np.float32))
        p0 = q.copy()
        m, v = np.zeros_like(q), np.zeros_like(q)
        for k in range(1, n + 1):
            _, g = net.gradients(X, T)
            net.train_step(X, T, lr=lr, beta1=b1, beta2=b2)
            q, m, v = O.adam_step(q, g.astype(np.float64), m, v, k, lr, b1, b2)
            d = float(np.abs(net.params() - q).max())
            worst = max(worst, d / lr)
            assert d < 1e-3 * lr, (n, k, d)
        moved = max(moved, float(np.abs(q - p0).max()))
        assert np.abs(q - p0).max() > 0.5 * n * lr
    print(f"Adam: 16 steps, largest parameter difference {worst:.2e} of the learning rate; "
          f"largest move {moved:.2e}", flush=True)
    net.close()


def test_training_reduces_a_smooth_loss(mlp):
    from paper_2002_04353_amd import surrogate as S
    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, (512, 5)).astype(np.float32)
    F = rng.standard_normal((5, 256))
    Y = np.sin(1.3 * X @ F).astype(np.float32)
    net = mlp.MLP(WIDTHS, 512, stream=0)
    net.set_params(S.glorot(WIDTHS, 0))
    losses = [net.train_step(X[i % 4 * 128:(i % 4 + 1) * 128], Y[i % 4 * 128:(i % 4 + 1) * 128], lr=2e-3)
              for i in range(600)]
    print(f"loss {losses[0]:.3f} -> {np.mean(losses[-8:]):.4f}", flush=True)
    assert np.mean(losses[-8:]) < losses[0] / 20
    net.close()


def test_surrogate_against_solver(mlp):
    """Train on solver histories of 48 cases, evaluate on 8 held-out cases: the
    network must beat what the method offers without it (the training mean,
    the nearest training case, an affine fit in the parameters) and answer far
    faster than the solver; outside the training box it must hand the query
    to the solver."""
    from paper_2002_04353_amd import cases
    from paper_2002_04353_amd import surrogate as S
    steps = 512
    mesh = cases.ensemble(n_cases=1, n_min=20_000, seed=21, shared_mesh=True)["meshes"][0]
    print(f"mesh {mesh.n_nodes} nodes", flush=True)
    train = cases.ensemble(n_cases=48, n_min=20_000, seed=22, shared_mesh=True)["motion"]
    test = cases.ensemble(n_cases=8, n_min=20_000, seed=23, shared_mesh=True)["motion"]
    Ytr, t_train = S.solver_histories(mesh, train, steps)
    Yte, t_test = S.solver_histories(mesh, test, steps)
    print(f"solver: {t_train:.2f} s for 48 cases, {t_test:.2f} s for 8", flush=True)
    assert np.isfinite(Ytr).all() and np.isfinite(Yte).all()
    sur = S.Surrogate(mesh, steps, max_batch=64)
    losses = sur.fit(S.scale_params(train), Ytr, iters=1500, batch=48)
    rms = sur.validate(test, Yte)
    base = {k: S.rms_cl_cm(v, Yte)
            for k, v in S.baselines(S.scale_params(train), Ytr, S.scale_params(test)).items()}
    t0 = time.perf_counter()
    P = sur.predict(S.scale_params(test))
    t_pred = time.perf_counter() - t0
    print(f"train loss {losses[0]:.3f} -> {losses[-1]:.4f}; held-out RMS cl {rms[0]:.4f} cm {rms[1]:.4f}; "
          f"without the network: " + ", ".join(f"{k} cl {v[0]:.4f} cm {v[1]:.4f}" for k, v in base.items()) +
          f"; predict {t_pred * 1e3:.2f} ms vs solver {t_test * 1e3:.0f} ms", flush=True)
    assert P.shape == Yte.shape
    # the gain over the method without the network: below the mean prediction
    # by a margin, and below the nearest training case and the affine fit
    assert rms[0] < 0.7 * base["mean"][0] and rms[1] < 0.7 * base["mean"][1]
    for k in ("nearest", "linear"):
        assert rms[0] < base[k][0] and rms[1] < base[k][1], k
    assert t_test / t_pred > 50
    # outside the training box: the solver answers
    far = test[:2].copy()
    far[:, 0] = 0.75  # Ma beyond the range the network was trained on
    Yf, who = sur.predict_or_solve(far)
    assert who == "solver"
    Yr, _ = S.solver_histories(mesh, far, steps)
    np.testing.assert_array_equal(Yf, Yr)
    _, who = sur.predict_or_solve(test[:2])
    assert who == "surrogate"
    sur.close()
