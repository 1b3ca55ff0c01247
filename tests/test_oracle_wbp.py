"""Pins for the oracle's weighted (unrolled) BP and its hand-written adjoint:
unit weights reproduce plain min-sum BP, and the reverse-mode gradient agrees
with FP64 central differences and with torch autograd of an independent
unrolled implementation."""
import numpy as np
import pytest
import torch

import synth

S_PRIOR = 2.0 ** 60


def _setup(orc, N, K, F, seed, snr=1.5):
    code = orc.construct(N, K, 2.5)
    msg = synth.message_bits(seed, F, K)
    _, x = orc.encode(code, msg)
    return code, synth.awgn_llr(x, snr, K, seed=seed)


def test_unit_weights_are_plain_bp(orc):
    code, llr = _setup(orc, 256, 128, 6, 1)
    T = 7
    w = np.ones((T, 8, 2, 256))
    out = orc.wbp_forward(code, llr, w, orc.WbpParams(fp32=True))
    for f in range(6):
        L, R = orc.bp_run(llr[f], code.frozen, T, fp32=True)
        info = code.info_idx
        np.testing.assert_array_equal(out[f, info], L[8, info])
        assert np.array_equal(out[f, info] < 0, (L[8, info] + R[8, info]) < 0)


def test_unit_weights_lastk_match_decoder(orc):
    code, llr = _setup(orc, 256, 128, 4, 2)
    T = 9
    w = np.ones((T, 8, 2, 256))
    out = orc.wbp_forward(code, llr, w, orc.WbpParams(pp_mode=orc.PP_LASTK, k=3, T_ev=4, Q=4,
                                                      seed=3, fp32=True))
    r = orc.decode(code, llr, orc.DecodeParams(max_iter=T, stop=orc.STOP_NONE,
                                               pp_mode=orc.PP_LASTK, k=3, T=4, Q=4, seed=3),
                   soft=True)
    info = code.info_idx
    np.testing.assert_array_equal(out[:, info], r.soft_u[:, info])


def _loss(orc, code, llr, w, p, g):
    return float((orc.wbp_forward(code, llr, w, p) * g).sum())


@pytest.mark.parametrize("T,pp", [(2, False), (3, False), (3, True)])
def test_gradient_central_differences(orc, T, pp):
    N, n = 16, 4
    code, llr = _setup(orc, N, 8, 3, 4 + T)
    rng = np.random.default_rng(T)
    w = rng.uniform(0.6, 1.4, (T, n, 2, N))
    g = rng.normal(size=(3, N))
    g[:, code.frozen.astype(bool)] = 0.0       # loss only on information positions
    p = (orc.WbpParams(pp_mode=orc.PP_LASTK, k=2, T_ev=1, Q=2, seed=5) if pp
         else orc.WbpParams())
    gw, gl = orc.wbp_backward(code, llr, w, p, g, want_llr_grad=True)
    h = 1e-6
    idx = rng.choice(w.size, 60, replace=False)
    flat = w.reshape(-1)
    for i in idx:
        wp = flat.copy(); wp[i] += h
        wm = flat.copy(); wm[i] -= h
        fd = (_loss(orc, code, llr, wp.reshape(w.shape), p, g)
              - _loss(orc, code, llr, wm.reshape(w.shape), p, g)) / (2 * h)
        assert gw.reshape(-1)[i] == pytest.approx(fd, rel=1e-6, abs=1e-6)
    # weights of the last R sweep never reach the output
    assert np.all(gw[T - 1, :, 1] == 0.0)


def _ms(x, y):
    sx = torch.where(torch.signbit(x), -1.0, 1.0)
    sy = torch.where(torch.signbit(y), -1.0, 1.0)
    return torch.where(x.abs() <= y.abs(), sy * x, sx * y)


class _AbsMul(torch.autograd.Function):
    """w * x whose backward uses the magnitudes of the local derivatives."""

    @staticmethod
    def forward(ctx, w, x):
        ctx.save_for_backward(w, x)
        return w * x

    @staticmethod
    def backward(ctx, g):
        w, x = ctx.saved_tensors
        return g.abs() * x.abs(), g.abs() * w.abs()


class _AbsMs(torch.autograd.Function):
    """Min-sum whose backward routes the magnitude of the adjoint to the
    smaller input (ties to the first), as the derivative's magnitude is 1."""

    @staticmethod
    def forward(ctx, x, y):
        ctx.save_for_backward(x, y)
        return _ms(x, y)

    @staticmethod
    def backward(ctx, g):
        x, y = ctx.saved_tensors
        first = x.abs() <= y.abs()
        return torch.where(first, g.abs(), 0.0), torch.where(first, 0.0, g.abs())


def _torch_wbp(llr, frozen, w, pool_orders, k, T_ev, absolute=False):
    """Independent unrolled weighted min-sum BP in torch (float64), rows
    vectorised.  absolute=True: the same forward values, with a backward
    whose every local derivative is replaced by its magnitude."""
    F, N = llr.shape
    T, n = w.shape[0], w.shape[1]
    prior = torch.where(torch.as_tensor(frozen.astype(bool)), torch.tensor(S_PRIOR, dtype=torch.float64),
                        torch.tensor(0.0, dtype=torch.float64))
    ms = _AbsMs.apply if absolute else _ms
    mul = _AbsMul.apply if absolute else torch.mul

    R = [torch.zeros(F, N, dtype=torch.float64) for _ in range(n + 1)]
    R[n] = prior.expand(F, N)
    Lc = torch.as_tensor(llr, dtype=torch.float64)
    qcur = 0
    for t in range(T):
        q = (t // T_ev) % len(pool_orders) if pool_orders is not None else 0
        if t > 0 and q != qcur:
            for lev in range(n - k + 1, n):
                R[lev] = torch.zeros(F, N, dtype=torch.float64)
        qcur = q
        order = pool_orders[q] if pool_orders is not None else list(range(n))
        # weight index: the row for stages outside the permuted range, the row's
        # position in the drawing of the active trellis inside it
        drawn = torch.tensor([sum(((j >> int(order[s])) & 1) << s for s in range(n))
                              for j in range(N)])
        ident = torch.arange(N)
        L = [Lc] + [None] * n
        for s in range(1, n + 1):
            b = int(order[s - 1])
            top = torch.tensor([j for j in range(N) if not (j >> b) & 1])
            bot = top | (1 << b)
            pos = drawn if (k and s > n - k) else ident
            l1, l2 = L[s - 1][:, top], L[s - 1][:, bot]
            r1, r2 = R[s][:, top], R[s][:, bot]
            out = torch.zeros(F, N, dtype=torch.float64)
            out = out.index_put((torch.arange(F)[:, None], top[None, :]),
                                mul(w[t, s - 1, 0, pos[top]], ms(l1, l2 + r2)))
            out = out.index_put((torch.arange(F)[:, None], bot[None, :]),
                                mul(w[t, s - 1, 0, pos[bot]], ms(r1, l1)) + l2)
            L[s] = out
        if t == T - 1:
            return L[n] + R[n]
        newR = [None] * (n + 1)
        newR[n] = R[n]
        for s in range(n, 0, -1):
            b = int(order[s - 1])
            top = torch.tensor([j for j in range(N) if not (j >> b) & 1])
            bot = top | (1 << b)
            pos = drawn if (k and s > n - k) else ident
            l1, l2 = L[s - 1][:, top], L[s - 1][:, bot]
            r1, r2 = newR[s][:, top], newR[s][:, bot]
            out = torch.zeros(F, N, dtype=torch.float64)
            out = out.index_put((torch.arange(F)[:, None], top[None, :]),
                                mul(w[t, s - 1, 1, pos[top]], ms(r1, l2 + r2)))
            out = out.index_put((torch.arange(F)[:, None], bot[None, :]),
                                mul(w[t, s - 1, 1, pos[bot]], ms(r1, l1)) + r2)
            newR[s - 1] = out
        R = newR


@pytest.mark.parametrize("N,T,pp", [(16, 3, False), (32, 4, True), (64, 3, False)])
def test_gradient_matches_torch_autograd(orc, N, T, pp):
    n = N.bit_length() - 1
    code, llr = _setup(orc, N, N // 2, 4, 20 + N)
    rng = np.random.default_rng(N)
    w = rng.uniform(0.6, 1.4, (T, n, 2, N))
    g = rng.normal(size=(4, N))
    g[:, code.frozen.astype(bool)] = 0.0
    if pp:
        p = orc.WbpParams(pp_mode=orc.PP_LASTK, k=3, T_ev=2, Q=3, seed=9)
        pool = orc.trellis_pool(n, 3, 3, seed=9)
        k, tev = 3, 2
    else:
        p = orc.WbpParams()
        pool, k, tev = None, 0, 1
    wt = torch.tensor(w, dtype=torch.float64, requires_grad=True)
    out = _torch_wbp(llr, code.frozen, wt, pool, k, tev)
    ref_out = orc.wbp_forward(code, llr, w, p)
    np.testing.assert_allclose(out.detach().numpy(), ref_out, rtol=1e-12, atol=0)
    (out * torch.as_tensor(g)).sum().backward()
    gw, _ = orc.wbp_backward(code, llr, w, p, g)
    np.testing.assert_allclose(gw, wt.grad.numpy(), rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("N,T,pp", [(16, 3, False), (32, 4, True), (64, 3, False)])
def test_gradient_magnitude_sums_match_torch(orc, N, T, pp):
    # the oracle's magnitude pass (the per-entry error scale of an FP32
    # adjoint) against torch autograd of the independent implementation with
    # every local derivative replaced by its magnitude; weights of both signs
    n = N.bit_length() - 1
    code, llr = _setup(orc, N, N // 2, 3, 40 + N)
    rng = np.random.default_rng(N + 1)
    w = rng.uniform(0.6, 1.4, (T, n, 2, N)) * rng.choice([-1.0, 1.0], (T, n, 2, N))
    g = rng.normal(size=(3, N))
    g[:, code.frozen.astype(bool)] = 0.0
    if pp:
        p = orc.WbpParams(pp_mode=orc.PP_LASTK, k=3, T_ev=2, Q=3, seed=9)
        pool, k, tev = orc.trellis_pool(n, 3, 3, seed=9), 3, 2
    else:
        p, pool, k, tev = orc.WbpParams(), None, 0, 1
    wt = torch.tensor(w, dtype=torch.float64, requires_grad=True)
    out = _torch_wbp(llr, code.frozen, wt, pool, k, tev, absolute=True)
    out.backward(torch.as_tensor(np.abs(g)))
    gw, _, ga = orc.wbp_backward(code, llr, w, p, g, want_abs=True)
    np.testing.assert_allclose(ga, wt.grad.numpy(), rtol=1e-10, atol=1e-10)
    # a sum of path magnitudes bounds the signed sum of the same paths, and
    # the gradient itself is unchanged by the extra pass
    assert np.all(np.abs(gw) <= ga * (1 + 1e-12))
    assert np.array_equal(gw, orc.wbp_backward(code, llr, w, p, g)[0])
    assert np.count_nonzero(ga) > 0.1 * ga.size
