"""The learned surrogate of the grid convolution on the GPU, through the C ABI:
the network's forward pass and its gradients against the plain FP64 network
of the oracle (oracle/surrogate.py) on a film grid of several tiles with
ragged ends, the synthetic textures, training, and the AIM-judged LLG loop
with its fallback."""
import numpy as np
import pytest

from oracle import surrogate as S
from paper_2409_13958_amd import meshgen as mg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2409_13958_amd import binding as B

C = 32


def bf16_round(a):
    """Round to the nearest BF16 value (ties to even), as the library does."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32)


def film(grid=(40, 24, 6)):
    """A film whose AIM grid spans two x tiles (32 + 8) and three y tiles of
    the kernels, six planes thick."""
    return mg.kuhn_box((20, 12, 2), 2e-9, periodic=0b011, jitter=0.1, seed=11, grid=grid)


def widths(depth):
    return [1] + [C] * (depth - 1) + [1]


def random_params(rng, depth, bias_sd=0.1):
    ps = []
    w = widths(depth)
    for l in range(depth):
        ci, co = w[l], w[l + 1]
        gain = 2.0 if l + 1 < depth else 1.0
        W = bf16_round(rng.standard_normal((co, ci, 3, 3, 3)) * np.sqrt(gain / (27 * ci)))
        b = (bias_sd * rng.standard_normal(co)).astype(np.float32)
        ps.append((W.astype(np.float64), b.astype(np.float64)))
    return ps


def gap_bias(zc, lo, hi):
    """minus the midpoint of the widest gap between consecutive sorted values
    of zc within the quantiles lo..hi"""
    v = np.sort(zc.ravel())
    i0, i1 = int(lo * v.size), int(hi * v.size)
    k = int(np.argmax(np.diff(v[i0:i1 + 1])))
    return -0.5 * (v[i0 + k] + v[i0 + k + 1])


def flat(ps):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in ps]).astype(np.float32)


def unflat(vec, depth):
    out, k = [], 0
    w = widths(depth)
    for l in range(depth):
        ci, co = w[l], w[l + 1]
        nW = co * ci * 27
        out.append((vec[k:k + nW].reshape(co, ci, 3, 3, 3), vec[k + nW:k + nW + co]))
        k += nW + co
    return out


@pytest.fixture(scope="module")
def ctx():
    c = B.Context.from_problem(film(), device=0)
    yield c
    c.close()


@pytest.mark.parametrize("bf16_act", [False, True])
def test_forward_matches_oracle(ctx, bf16_act):
    """Six layers, scales 1/2 and 2 (powers of two, exact): the FP32-accurate
    form within 1e-5 of the FP64 network (relative to the largest output);
    the BF16-activation form within 1e-2 in relative L2 (each of the four
    matrix-core layers rounds its inputs to 8 significant bits, 2^-9 relative,
    4 x 2^-9 < 1e-2)."""
    depth = 6
    ctx.surrogate_init(depth, seed=3, bf16_activations=bf16_act)
    shape = ctx._grid_shape()
    rng = np.random.default_rng(5)
    ps = random_params(rng, depth)
    ctx.surrogate_set_params(flat(ps), scales=(0.5, 2.0))
    Q = rng.standard_normal(shape).astype(np.float32)
    ref = S.forward(0.5 * Q.astype(np.float64)[None], ps)[0][0] * 2.0
    qg = torch.tensor(Q, device="cuda")
    ug = torch.empty_like(qg)
    print(f"[gpu surrogate] forward grid {shape} bf16_act={bf16_act}", flush=True)
    ctx.surrogate_apply(qg, ug)
    U = ug.cpu().numpy().astype(np.float64)
    errmax = np.abs(U - ref).max() / np.abs(ref).max()
    errl2 = np.linalg.norm(U - ref) / np.linalg.norm(ref)
    print(f"[gpu surrogate] forward: max {errmax:.2e}, rel L2 {errl2:.2e}", flush=True)
    if bf16_act:
        assert errl2 <= 1e-2
    else:
        assert errmax <= 1e-5
    # in place (the buffer holding Q receives U)
    qg2 = torch.tensor(Q, device="cuda")
    ctx.surrogate_apply(qg2, qg2)
    assert torch.equal(qg2, ug)


@pytest.mark.parametrize("bf16_act", [False, True])
def test_forward_odd_thickness(bf16_act):
    """Grid 36 x 16 x 5: a ragged x tile of 4 points, and an odd number of
    planes, so that the last workgroup of the matrix-core layer computes one
    plane instead of two; bars as above."""
    prob = mg.kuhn_box((18, 8, 2), 2e-9, periodic=0b011, jitter=0.1, seed=13, grid=(36, 16, 5))
    c = B.Context.from_problem(prob, device=0)
    try:
        depth = 5
        c.surrogate_init(depth, seed=2, bf16_activations=bf16_act)
        shape = c._grid_shape()
        assert shape == (5, 16, 36)
        rng = np.random.default_rng(15)
        ps = random_params(rng, depth)
        c.surrogate_set_params(flat(ps), scales=(1.0, 1.0))
        Q = rng.standard_normal(shape).astype(np.float32)
        ref = S.forward(Q.astype(np.float64)[None], ps)[0][0]
        qg = torch.tensor(Q, device="cuda")
        ug = torch.empty_like(qg)
        print(f"[gpu surrogate] forward grid {shape} bf16_act={bf16_act}", flush=True)
        c.surrogate_apply(qg, ug)
        U = ug.cpu().numpy().astype(np.float64)
        errmax = np.abs(U - ref).max() / np.abs(ref).max()
        errl2 = np.linalg.norm(U - ref) / np.linalg.norm(ref)
        print(f"[gpu surrogate] forward: max {errmax:.2e}, rel L2 {errl2:.2e}", flush=True)
        assert (errl2 <= 1e-2) if bf16_act else (errmax <= 1e-5)
    finally:
        c.close()


def test_grid_narrower_than_a_tile():
    """The 20 x 20 x 2 nm film's grid, 16 x 16 x 4: narrower than a kernel
    tile (32 points), so the staged halo wraps around the period more than
    once and half of every tile lies outside the grid. Forward and gradients
    of a three-layer network against the oracle, ReLU margins as in the
    gradient test below."""
    c = B.Context.from_problem(mg.film_c1(), device=0)
    try:
        depth = 3
        c.surrogate_init(depth, seed=7)
        shape = c._grid_shape()
        assert shape == (4, 16, 16)
        rng = np.random.default_rng(17)
        ps = random_params(rng, depth, bias_sd=0.0)
        Q = rng.standard_normal(shape).astype(np.float32)
        h = Q.astype(np.float64)[None]
        margins = []
        for l in range(depth):
            W, _ = ps[l]
            z = S.layer(h, W, np.zeros(W.shape[0]))
            sd = z.reshape(z.shape[0], -1).std(axis=1)
            b = np.array([gap_bias(z[k], *((0.02, 0.2) if rng.random() < 0.5 else (0.8, 0.98)))
                          for k in range(W.shape[0])]).astype(np.float32).astype(np.float64)
            ps[l] = (W, b)
            z = z + b[:, None, None, None]
            if l + 1 < depth:
                margins.append(np.min(np.abs(z).reshape(z.shape[0], -1) / sd[:, None]))
                h = np.maximum(z, 0.0)
        assert min(margins) > 1e-4, margins
        c.surrogate_set_params(flat(ps), scales=(1.0, 1.0))
        qg = torch.tensor(Q, device="cuda")
        ug = torch.empty_like(qg)
        print(f"[gpu surrogate] grid {shape}: forward and gradients", flush=True)
        c.surrogate_apply(qg, ug)
        ref = S.forward(Q.astype(np.float64)[None], ps)[0][0]
        U = ug.cpu().numpy().astype(np.float64)
        assert np.abs(U - ref).max() <= 1e-5 * np.abs(ref).max()
        T = rng.standard_normal(shape).astype(np.float32)
        loss_o, grads_o = S.loss_and_grads(Q.astype(np.float64)[None],
                                           T.astype(np.float64)[None], ps)
        loss_k, gk = c.surrogate_loss_grad(qg, torch.tensor(T, device="cuda"))
        assert abs(loss_k - loss_o) <= 1e-5 * loss_o
        for (gW, gb), (kW, kb) in zip(grads_o, unflat(gk.astype(np.float64), depth)):
            assert np.abs(kW - gW).max() <= 1e-4 * np.abs(gW).max()
            assert np.abs(kb - gb).max() <= 1e-4 * np.abs(gb).max()
    finally:
        c.close()


@pytest.mark.parametrize("depth", [6, 2])
def test_gradients_match_oracle(ctx, depth):
    """Loss and every parameter's gradient against the oracle's
    back-propagation. Each hidden channel's bias puts zero in the middle of
    the widest gap between its sorted convolution values inside a quantile
    window (2-20 % or 80-98 %, random), so that the ReLU is active on a
    varying set of points in every channel, and the test first checks, on the
    oracle alone, that no pre-activation lies within 1e-4 of its channel's
    spread of zero, far outside the kernel's forward error (~1e-6): so both
    sides take the same ReLU decisions. Depth 2 is the degenerate network
    with no matrix-core layer (first layer straight into the last)."""
    ctx.surrogate_init(depth, seed=4)
    shape = ctx._grid_shape()
    rng = np.random.default_rng(9)
    ps = random_params(rng, depth, bias_sd=0.0)
    Q = rng.standard_normal(shape).astype(np.float32)
    h = Q.astype(np.float64)[None]
    margins = []
    for l in range(depth):
        W, _ = ps[l]
        z = S.layer(h, W, np.zeros(W.shape[0]))
        sd = z.reshape(z.shape[0], -1).std(axis=1)
        b = np.array([gap_bias(z[c], *((0.02, 0.2) if rng.random() < 0.5 else (0.8, 0.98)))
                      for c in range(W.shape[0])])
        b = b.astype(np.float32).astype(np.float64)
        ps[l] = (W, b)
        z = z + b[:, None, None, None]
        if l + 1 < depth:
            margins.append(np.min(np.abs(z).reshape(z.shape[0], -1) / sd[:, None]))
            h = np.maximum(z, 0.0)
    assert min(margins) > 1e-4, margins
    T = rng.standard_normal(shape).astype(np.float32)
    loss_o, grads_o = S.loss_and_grads(Q.astype(np.float64)[None], T.astype(np.float64)[None], ps)
    ctx.surrogate_set_params(flat(ps), scales=(1.0, 1.0))
    print(f"[gpu surrogate] gradients grid {shape}", flush=True)
    loss_k, gk = ctx.surrogate_loss_grad(torch.tensor(Q, device="cuda"), torch.tensor(T, device="cuda"))
    assert abs(loss_k - loss_o) <= 1e-5 * loss_o
    for l, ((gW, gb), (kW, kb)) in enumerate(zip(grads_o, unflat(gk.astype(np.float64), depth))):
        eW = np.abs(kW - gW).max() / np.abs(gW).max()
        eb = np.abs(kb - gb).max() / np.abs(gb).max()
        print(f"[gpu surrogate] layer {l}: dW max {eW:.2e}, db max {eb:.2e}", flush=True)
        assert eW <= 1e-4 and eb <= 1e-4, (l, eW, eb)


def test_textures(ctx):
    n = ctx.n
    m = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    out = []
    for kind in (0, 1, 2):
        ctx.surrogate_init(2, seed=0)
        ctx.surrogate_texture(m, kind, seed=21)
        a = m.cpu().numpy()
        assert np.abs(np.linalg.norm(a, axis=1) - 1.0).max() < 1e-12
        ctx.surrogate_texture(m, kind, seed=21)
        assert np.array_equal(m.cpu().numpy(), a)
        ctx.surrogate_texture(m, kind, seed=22)
        assert not np.array_equal(m.cpu().numpy(), a)
        out.append(a)
    rnd, vtx, wall = out
    assert np.abs(rnd.mean(axis=0)).max() < 0.1
    assert abs((rnd[:, 2] ** 2).mean() - 1.0 / 3.0) < 0.05
    # a vortex: m_z of one sign (the polarity), small away from the core
    assert (vtx[:, 2] >= 0).all() or (vtx[:, 2] <= 0).all()
    assert np.abs(vtx[:, 2]).mean() < 0.5
    # two domains: some component changes sign across the cell
    assert (wall.min(axis=0) < -0.5).any() and (wall.max(axis=0) > 0.5).any()


def test_training_lowers_the_loss():
    prob = mg.kuhn_box((16, 16, 2), 2e-9, periodic=0b011, jitter=0.1, seed=12, grid=(32, 32, 4))
    c = B.Context.from_problem(prob, device=0)
    try:
        c.surrogate_init(6, seed=1)
        print("[gpu surrogate] training 80 pairs", flush=True)
        log = c.surrogate_train(80, lr=2e-3, seed=2, kinds=0b110)
        assert np.isfinite(log).all()
        first, last = log[:4].mean(), log[-16:].mean()
        print(f"[gpu surrogate] loss {first:.3e} -> {last:.3e}", flush=True)
        assert last < 0.5 * first
        p, (s_in, s_out) = c.surrogate_get_params()
        assert s_in > 0 and s_out > 0 and np.isfinite(p).all()
    finally:
        c.close()


def test_training_is_reproducible(ctx):
    """The same initialisation and pairs give the same parameters and losses,
    bit for bit (fixed-order reductions, no atomics)."""
    runs = []
    for _ in range(2):
        ctx.surrogate_init(4, seed=12)
        log = ctx.surrogate_train(6, lr=1e-3, seed=5)
        p, sc = ctx.surrogate_get_params()
        runs.append((log, p, sc))
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1])
    assert runs[0][2] == runs[1][2]
    ctx.surrogate_init(4, seed=12)
    other = ctx.surrogate_train(6, lr=1e-3, seed=6)
    assert not np.array_equal(other, runs[0][0])


def test_judged_llg_and_fallback(ctx):
    n = ctx.n
    ctx.surrogate_init(4, seed=6)
    ctx.surrogate_train(4, lr=1e-3, seed=1)
    m0 = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    ctx.surrogate_texture(m0, 1, seed=5)
    dt, alpha, steps, every = 1e-13, 0.5, 12, 5
    # the error the judge reports at the first check, recomputed from H_ms
    m32 = m0.float()
    ha = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    hs = torch.empty_like(ha)
    ctx.heff(m32, ha, terms=B.TERM_MS)
    ctx.surrogate_enable(True)
    ctx.heff(m32, hs, terms=B.TERM_MS)
    ctx.surrogate_enable(False)
    err0 = float(torch.linalg.norm((hs - ha).double()) / torch.linalg.norm(ha.double()))
    print(f"[gpu surrogate] judged LLG: initial field error {err0:.3e}", flush=True)
    # a tolerance no error meets: fallback before the first step, then the
    # plain trajectory bit for bit
    m_a = m0.clone()
    rep = ctx.llg_step_judged(m_a, dt, alpha, steps, check_every=every, tol=0.0)
    assert rep["fallback_step"] == 0 and rep["checks"] == 1
    assert abs(rep["last_error"] - err0) <= 1e-6 * err0
    m_b = m0.clone()
    ctx.llg_step(m_b, dt, alpha, steps)
    assert torch.equal(m_a, m_b)
    # a tolerance every error meets: the surrogate all the way, checked before
    # steps 0, 5, 10; the same trajectory as the surrogate-enabled stepper
    m_c = m0.clone()
    rep = ctx.llg_step_judged(m_c, dt, alpha, steps, check_every=every, tol=1e9)
    assert rep["fallback_step"] == -1 and rep["checks"] == 3
    m_d = m0.clone()
    ctx.surrogate_enable(True)
    ctx.llg_step(m_d, dt, alpha, steps)
    ctx.surrogate_enable(False)
    assert torch.equal(m_c, m_d)
    assert not torch.equal(m_c, m_b)
    assert np.abs(torch.linalg.norm(m_c, dim=1).cpu().numpy() - 1.0).max() < 1e-12


def test_step_graph_follows_the_surrogate(ctx):
    """The captured RK4 step is captured again when the surrogate is switched
    on or off, re-created or retrained, and replays what pmfem_llg_step does
    in each state, bit for bit."""
    n = ctx.n
    m0 = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    ctx.surrogate_init(3, seed=8)
    ctx.surrogate_train(2, lr=1e-3, seed=3)
    ctx.surrogate_texture(m0, 2, seed=9)
    dt, alpha = 1e-13, 0.5

    def both(on):
        ctx.surrogate_enable(on)
        a, b = m0.clone(), m0.clone()
        ctx.llg_step_graph(a, dt, alpha, 3)
        ctx.llg_step(b, dt, alpha, 3)
        ctx.surrogate_enable(False)
        assert torch.equal(a, b)
        return a

    plain = both(False)
    sur = both(True)
    assert not torch.equal(plain, sur)
    assert torch.equal(both(False), plain)
    # a new network (new buffers and weights) behind the same switch
    ctx.surrogate_init(3, seed=10)
    ctx.surrogate_train(2, lr=1e-3, seed=4)
    sur2 = both(True)
    assert not torch.equal(sur2, sur)


def test_surrogate_rejects_bad_use():
    prob = mg.film_c1()
    c = B.Context.from_problem(prob, device=0)
    try:
        with pytest.raises(B.PmfemError):
            c.surrogate_enable(True)             # before init
        with pytest.raises(B.PmfemError):
            c.surrogate_init(1)                  # depth below 2
        c.surrogate_init(3, seed=0)
        shape = c._grid_shape()
        q = torch.zeros(shape, device="cuda")
        with pytest.raises(B.PmfemError):
            c.surrogate_apply(q, q)              # scales unset
        with pytest.raises(B.PmfemError):
            c.surrogate_set_params(np.zeros(5, np.float32))
    finally:
        c.close()
    wire = B.Context.from_problem(mg.kuhn_box((4, 4, 8), 2e-9, periodic=0b100, grid=(8, 8, 16)),
                                  device=0)
    try:
        with pytest.raises(B.PmfemError):
            wire.surrogate_init(3)               # not a film
    finally:
        wire.close()
