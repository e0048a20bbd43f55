"""The learned Ewald surrogate on the GPU, through the C ABI.

* Training gradients (FP32 forward + backward kernels, fixed-order reduction)
  against the oracle's FP64 back-propagation: max-normalised 1e-5.
* Matrix-core inference (FP16 inputs, FP32 accumulation) against the oracle's
  FP64 forward of the same weights, within a first-order bound of that
  arithmetic propagated through the layers (below).
* The device FP64 Ewald series and table lookups at arbitrary offsets against
  the oracle: 1e-12 of each channel's largest value.
* Training on FP64 series values: the loss falls, training is reproducible bit
  for bit, and the trained network beats a smaller table (9^3 points x 10
  channels, ~29 KB in FP32, vs 9226 FP32 parameters, ~37 KB).
* The walk with the surrogate against the table walk on the same lists,
  within the held-out error carried through the sum over the list and within
  1e-4 of the largest |Phi| and |a| (the surrogate's accuracy budget); without
  an accepted surrogate the walk is the table walk, bit for bit.
"""
import numpy as np
import pytest

import oracle
import paper_1708_06142_amd as ot
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U16 = 2.0 ** -11        # unit roundoff of FP16
G32 = 64 * 2.0 ** -24   # FP32 accumulation of a 64-term sum
LACT = 1.21             # max |f'| of the activation z S(z)
TINY = 2.0 ** -14       # smallest normal FP16 value


def small(W):
    """|W| where FP16 holds W below its normal range, else 0."""
    return np.where(np.abs(W) < TINY, np.abs(W), 0.0)

BOXES = {"3p": ((1, 1, 1), 1.0, (1, 1, 1)), "2p1i": ((1, 1, 4), 1.0, (1, 1, 0))}


def solver(name, **kw):
    nroot, rs, bc = BOXES[name]
    return ot.Solver(nroot=nroot, root_size=rs, bc=bc, **kw)


def extent(name):
    """Folded domain of the correction: half the box in periodic axes, 2 Lx in
    the isolated axis of 2P1I."""
    return np.array([0.5, 0.5, 0.5]) if name == "3p" else np.array([0.5, 0.5, 2.0])


NO = ot.MLP_NOUT


def unpack(p):
    o, out = 0, []
    for shape in ((64, 3), (64,), (64, 64), (64,), (64, 64), (64,), (NO, 64), (NO,)):
        k = int(np.prod(shape))
        out.append(p[o:o + k].reshape(shape))
        o += k
    return out


def act(z):
    t = np.clip(z / 6 + 0.5, 0, 1)
    return z * t * t * (3 - 2 * t)


def unfold(y, d):
    """Signs of the ten channels at offsets d from their values at |d|."""
    s = np.where(d < 0, -1.0, 1.0)
    y = y.copy()
    y[:, 1:4] *= s
    y[:, 7] *= s[:, 0] * s[:, 1]
    y[:, 8] *= s[:, 0] * s[:, 2]
    y[:, 9] *= s[:, 1] * s[:, 2]
    return y


def forward_with_bound(p, norm, d):
    """FP64 output (the ten channels, signed) of the network at offsets d, from the
    oracle's forward pass, and a first-order bound of the error of evaluating
    it with FP16 weights and activations and FP32 sums: per layer
    |dz| <= (U16 + G32) sum |W| (|h| + |dh|) + sum |W| |dh|, and after the
    activation |dh| <= LACT |dz| + U16 (|h| + LACT |dz|).  Inputs and biases
    are split into FP16 high and low parts on the device (error O(U16^2)).
    Values below FP16's smallest normal (2^-14) may lose all precision, which
    adds their whole product to the bound."""
    p = np.asarray(p, np.float64)
    ext, mu, sig = norm[:3], norm[3:3 + NO], norm[3 + NO:3 + 2 * NO]
    u = np.abs(d)
    y = oracle.mlp_forward(p, 2 * u / ext - 1) * sig + mu
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(p)
    W1s = W1 * (2 / ext)
    z = u @ W1s.T + (b1 - W1.sum(1))
    dz = (U16 + G32) * (np.abs(u) @ np.abs(W1s).T) + 4 * U16 ** 2 * (np.abs(b1) + np.abs(W1).sum(1))
    dz += np.abs(u) @ small(W1s).T

    def layer(h, dh, W, b):
        a = np.abs(h) + dh
        return ((U16 + G32) * (a @ np.abs(W).T) + dh @ np.abs(W).T + a @ small(W).T
                + 4 * U16 ** 2 * np.abs(b))

    for W, b in ((W2, b2), (W3, b3)):
        h = act(z)
        dh = LACT * dz + U16 * (np.abs(h) + LACT * dz) + TINY
        z = h @ W.T + b
        dz = layer(h, dh, W, b)
    h = act(z)
    dh = LACT * dz + U16 * (np.abs(h) + LACT * dz) + TINY
    bound = layer(h, dh, W4 * sig[:, None], b4 * sig) + 4 * U16 ** 2 * np.abs(mu)
    return unfold(y, d), bound


def random_params(seed):
    rng = np.random.default_rng(seed)
    p = np.zeros(ot.MLP_NPARAM, np.float32)
    W1, b1, W2, b2, W3, b3, W4, b4 = (slice(0, 192), slice(192, 256), slice(256, 4352), slice(4352, 4416),
                                      slice(4416, 8512), slice(8512, 8576), slice(8576, 8576 + 64 * NO),
                                      slice(8576 + 64 * NO, 8576 + 65 * NO))
    p[W1] = rng.uniform(-1, 1, 192) * np.sqrt(6 / 3)
    for s in (W2, W3, W4):
        p[s] = rng.uniform(-1, 1, s.stop - s.start) * np.sqrt(6 / 64)
    for s in (b1, b2, b3, b4):
        p[s] = rng.uniform(-0.5, 0.5, s.stop - s.start)
    return p


def offsets(name, n, seed, signed=True):
    rng = np.random.default_rng(seed)
    d = rng.uniform(0, 1, (n, 3)) * extent(name)
    if signed:
        d *= rng.choice([-1.0, 1.0], (n, 3))
    d[:3] = 0.0          # offsets on the axes and at the origin of the fold
    d[0, :] = [0.0, 0.0, 0.3]
    d[1, :] = [extent(name)[0], 0.0, 0.0]
    return d


def dev(a, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)


# ------------------------------------------------------------- gradients
@pytest.mark.parametrize("batch", [32, 96, 512])
def test_gradient_vs_oracle(batch):
    s = solver("3p")
    rng = np.random.default_rng(batch)
    p = random_params(batch)
    x = rng.uniform(-1, 1, (batch, 3)).astype(np.float32)
    t = rng.normal(size=(batch, NO)).astype(np.float32)
    g = torch.empty(ot.MLP_NPARAM, dtype=torch.float32, device="cuda")
    loss = s.mlp_grad(dev(p, torch.float32), dev(x, torch.float32), dev(t, torch.float32), g)
    lr, gr = oracle.mlp_grad(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    gg = g.cpu().numpy().astype(np.float64)
    err = np.abs(gg - gr).max() / np.abs(gr).max()
    print(f"batch {batch}: loss {loss:.6g} (oracle {lr:.6g}), gradient error {err:.2e}")
    assert abs(loss - lr) <= 1e-5 * lr
    assert err <= 1e-5
    # every block of the parameter vector is covered
    for sl in (slice(0, 192), slice(192, 256), slice(4352, 4416), slice(8576, 8576 + 64 * NO),
               slice(8576 + 64 * NO, ot.MLP_NPARAM)):
        assert np.abs(gg[sl] - gr[sl]).max() <= 1e-5 * np.abs(gr).max()


@pytest.mark.parametrize("step", [1, 7])
def test_adam_step_vs_oracle(step):
    """One device training step (the trainer's kernels: FP32 gradient, then
    Adam with bias corrections for update index step) against the oracle's
    FP64 gradient and Adam step from the same parameters, moments and batch:
    parameters within 1e-6 (the updates are about lr = 1e-3), the moment
    estimates within 1e-5 of their largest value."""
    s = solver("3p")
    rng = np.random.default_rng(40 + step)
    batch, lr = 96, 1e-3
    p = random_params(50 + step)
    m = (1e-2 * rng.normal(size=p.size)).astype(np.float32)
    v = (1e-4 * rng.uniform(0.1, 1.0, p.size)).astype(np.float32)
    x = rng.uniform(-1, 1, (batch, 3)).astype(np.float32)
    t = rng.normal(size=(batch, NO)).astype(np.float32)
    pd, md, vd = (dev(a, torch.float32) for a in (p, m, v))
    loss = s.mlp_adam_step(pd, md, vd, dev(x, torch.float32), dev(t, torch.float32), lr, step)
    lr_, pr, mr, vr = oracle.mlp_adam(p.astype(np.float64), m.astype(np.float64), v.astype(np.float64),
                                      x.astype(np.float64), t.astype(np.float64), lr, step)
    got = [a.cpu().numpy().astype(np.float64) for a in (pd, md, vd)]
    ep = np.abs(got[0] - pr).max()
    em = np.abs(got[1] - mr).max() / np.abs(mr).max()
    ev = np.abs(got[2] - vr).max() / np.abs(vr).max()
    print(f"step {step}: loss {loss:.6g} (oracle {lr_:.6g}); |dP| {ep:.2e}, m {em:.2e}, v {ev:.2e}, "
          f"largest update {np.abs(pr - p).max():.2e}")
    assert abs(loss - lr_) <= 1e-5 * lr_
    assert np.abs(pr - p).max() > 1e-4  # the step moves the parameters
    assert ep <= 1e-6 and em <= 1e-5 and ev <= 1e-5
    with pytest.raises(ot.OTError, match="INVALID_ARG"):
        s.mlp_adam_step(pd, md, vd, dev(x, torch.float32), dev(t, torch.float32), lr, 0)


def test_gradient_is_deterministic():
    s = solver("3p")
    rng = np.random.default_rng(9)
    p = dev(random_params(9), torch.float32)
    x = dev(rng.uniform(-1, 1, (4096, 3)), torch.float32)
    t = dev(rng.normal(size=(4096, NO)), torch.float32)
    g1 = torch.empty(ot.MLP_NPARAM, dtype=torch.float32, device="cuda")
    g2 = torch.empty_like(g1)
    l1 = s.mlp_grad(p, x, t, g1)
    l2 = s.mlp_grad(p, x, t, g2)
    assert l1 == l2 and torch.equal(g1, g2)


def test_grad_rejects_bad_batch():
    s = solver("3p")
    g = torch.empty(ot.MLP_NPARAM, dtype=torch.float32, device="cuda")
    x = torch.zeros((40, 3), dtype=torch.float32, device="cuda")
    t = torch.zeros((40, NO), dtype=torch.float32, device="cuda")
    with pytest.raises(ot.OTError) as e:
        s.mlp_grad(g, x, t, g)
    assert e.value.status == ot.OT_ERR_INVALID_ARG


# ------------------------------------------------------------- inference
@pytest.mark.parametrize("name", list(BOXES))
def test_inference_vs_oracle_forward(name):
    s = solver(name, ewald_n=16)
    p = random_params(3)
    norm = np.concatenate([extent(name), [0.3, -0.2, 0.1, 1.5, 0.8, -1.1, 0.2, 0.6, -0.4, 0.9],
                           [2.0, 0.7, 1.3, 0.4, 3.0, 1.7, 0.9, 2.2, 0.5, 1.1]])
    s.mlp_set(p, norm, accept=False)
    n = 1000  # not a multiple of 32: a ragged last batch
    d = offsets(name, n, 11)
    out = torch.empty((n, NO), dtype=torch.float64, device="cuda")
    s.ewald_points("mlp", dev(d), out)
    y = out.cpu().numpy()
    ref, bound = forward_with_bound(p, norm, d)
    excess = (np.abs(y - ref) - bound).max()
    rel = np.abs(y - ref).max(0) / np.abs(ref).max(0)
    print(f"{name}: max error / channel max {rel}, max error / bound {(np.abs(y - ref) / bound).max():.3f}")
    assert excess <= 0, excess
    p2, n2 = s.mlp_get()
    assert np.array_equal(p2, p) and np.array_equal(n2, norm)


# ------------------------------------------------------------- series / table points
@pytest.mark.parametrize("name", list(BOXES))
def test_points_series_and_table_vs_oracle(name):
    nroot, rs, bc = BOXES[name]
    box = np.array(nroot, float) * rs
    s = solver(name, ewald_n=24)
    d = offsets(name, 300, 5)
    d = d[np.abs(d).sum(1) > 0]  # the series' correction is regular at 0 but keep to d != 0
    out = torch.empty((d.shape[0], NO), dtype=torch.float64, device="cuda")
    s.ewald_points("exact", dev(d), out)
    ref = oracle.ewald_eval(bc, box, d, correction=True)
    got = out.cpu().numpy()
    for ch in range(NO):
        assert np.abs(got[:, ch] - ref[:, ch]).max() <= 1e-12 * np.abs(ref[:, ch]).max(), ch
    s.ewald_points("table", dev(d), out)
    tab = oracle.ewald_table(bc, box, n=24)
    reft = oracle.ewald_table_lookup(bc, box, tab, d)[:, :4]
    # second derivatives: the nearest grid point's, signs restored
    ext = extent(name) if name == "3p" else np.array([0.5, 0.5, min(box[2], 2 * box[0])])
    step = ext / 23
    g = np.minimum(np.floor(np.abs(d) / step + 0.5).astype(int), 23)
    hn = np.zeros((d.shape[0], NO))
    hn[:, 4:] = tab[g[:, 2], g[:, 1], g[:, 0], 4:]
    reft = np.concatenate([reft, unfold(hn, d)[:, 4:]], 1)
    got = out.cpu().numpy()
    for ch in range(NO):
        assert np.abs(got[:, ch] - reft[:, ch]).max() <= 1e-12 * np.abs(reft[:, ch]).max(), ch


def test_points_need_a_surrogate():
    s = solver("3p", ewald_n=8)
    d = dev(np.full((4, 3), 0.1))
    out = torch.empty((4, NO), dtype=torch.float64, device="cuda")
    with pytest.raises(ot.OTError) as e:
        s.ewald_points("mlp", d, out)
    assert e.value.status == ot.OT_ERR_STATE


# ------------------------------------------------------------- training
TRAIN = dict(nval=50000)  # otherwise the library defaults (2^21 offsets, 100 epochs)


@pytest.fixture(scope="module")
def trained():
    out = {}
    for name in BOXES:
        s = solver(name, ewald_n=64, ewald="mlp")
        rep = s.mlp_train(**TRAIN)
        print(f"{name}: {rep}")
        out[name] = (s, rep)
    return out


@pytest.mark.parametrize("name", list(BOXES))
def test_training_reduces_loss(trained, name):
    _, rep = trained[name]
    assert rep["loss_last"] < 0.01 * rep["loss_first"], rep


@pytest.mark.parametrize("name", list(BOXES))
def test_gain_over_equal_memory_table(trained, name):
    """The surrogate against a table of the same memory (9^3 points) and the
    default 64^3 table, on the same held-out offsets, all against the series."""
    s, rep = trained[name]
    d = offsets(name, 20000, 21)
    dd = dev(d)
    out = torch.empty((d.shape[0], NO), dtype=torch.float64, device="cuda")
    s.ewald_points("exact", dd, out)
    ex = out.cpu().numpy()[:, :4]  # phi_c and A_c, the channels a 9^3 table looks up with its Taylor term
    scale = np.abs(ex).max(0)
    s.ewald_points("mlp", dd, out)
    e_mlp = (np.abs(out.cpu().numpy()[:, :4] - ex).max(0) / scale).max()
    s.ewald_points("table", dd, out)
    e_t64 = (np.abs(out.cpu().numpy()[:, :4] - ex).max(0) / scale).max()
    s9 = solver(name, ewald_n=9)
    s9.ewald_points("table", dd, out)
    e_t9 = (np.abs(out.cpu().numpy()[:, :4] - ex).max(0) / scale).max()
    print(f"{name}: max-normalised error: surrogate {e_mlp:.2e}, table 9^3 {e_t9:.2e}, table 64^3 {e_t64:.2e}")
    assert e_mlp < e_t9 / 3


def test_training_is_reproducible():
    cfg = dict(nsamples=1 << 14, epochs=3, batch=2048, nval=1000)
    a = solver("3p", ewald_n=16)
    b = solver("3p", ewald_n=16)
    ra, rb = a.mlp_train(**cfg), b.mlp_train(**cfg)
    pa, na = a.mlp_get()
    pb, nb = b.mlp_get()
    assert np.array_equal(pa, pb) and np.array_equal(na, nb)
    assert ra["loss_last"] == rb["loss_last"]
    c = solver("3p", ewald_n=16)
    c.mlp_train(seed=5, **cfg)
    assert not np.array_equal(c.mlp_get()[0], pa)


# ------------------------------------------------------------- walk
def lognormal32(bc, nroot=(1, 1, 1)):
    n = 32
    nb = n // 8
    level, coord = workloads.uniform_blocks(n)
    rng = np.random.default_rng(17)
    rho = rng.lognormal(0.0, 1.0, (nb ** 3, 8, 8, 8))
    if nroot != (1, 1, 1):
        level, coord, rho = [], [], []
        for z in range(nroot[2]):
            l, c = workloads.uniform_blocks(n)
            c = np.array(c).copy()
            c[:, 2] += z * nb
            level.append(l)
            coord.append(c)
            rho.append(rng.lognormal(0.0, 1.0, (nb ** 3, 8, 8, 8)))
        level, coord, rho = np.concatenate(level), np.concatenate(coord), np.concatenate(rho)
    return workloads.Grid(nroot, 1.0, (0, 0, 0), level, coord, rho, bc, "lognormal32")


GRIDS = {"3p": ((1, 1, 1), (1, 1, 1)), "2p1i": ((1, 1, 0), (1, 1, 4))}


def solve32(g, rho, mode, mlp=None, **kw):
    kw.setdefault("theta", 0.5)
    s = ot.Solver.for_grid(g, ewald_n=64, ewald=mode, **kw)
    if mlp is not None:
        s.mlp_set(*mlp, accept=True)
    s.build(rho)
    n = g.nb * 512
    out = [torch.empty(n, dtype=torch.float32, device="cuda"), torch.empty(3 * n, dtype=torch.float32, device="cuda")]
    if s.params.nside:
        npx = 12 * s.params.nside ** 2
        out += [torch.empty(n * npx, dtype=torch.float32, device="cuda"),
                torch.empty(n, dtype=torch.float32, device="cuda")]
    st = s.solve(*out)
    res = [o.cpu().numpy().astype(np.float64) for o in out]
    res[1] = res[1].reshape(3, -1)
    return res, st, s


def taylor_reach():
    """Largest per-axis offset of a cell from its group centre: half the
    64^3 table's smallest spacing (x: 0.5 / 63)."""
    return 0.5 * 0.5 / 63


@pytest.mark.parametrize("grid", ["lognormal32", "deep"])
@pytest.mark.parametrize("name", list(BOXES))
def test_walk_with_surrogate(trained, name, grid):
    """Same lists as the FP32 table walk.  Per pair the two differ by the
    network's error at the group centre, its second derivatives' error over
    the Taylor offset, and the Taylor remainders of both look-ups (each at
    most the table's own error): bounded by G M_total ((e_mlp + 2 e_table)
    max|phi_c| + 3 reach e_mlp max|A_c|) for Phi and likewise for a, a factor
    2 for the held-out maximum not being the global one.  And the accuracy
    budget: 1e-4 of max |Phi| and max |a|."""
    s_tr, rep = trained[name]
    params, norm = s_tr.mlp_get()
    nroot, _, bc = BOXES[name]
    g = lognormal32(bc, nroot) if grid == "lognormal32" else workloads.deep_amr(*GRIDS[name])
    rho = dev(g.rho.reshape(-1))
    (pt, at), st_t, s_t = solve32(g, rho, "table")
    (pm, am), st_m, s_m = solve32(g, rho, "mlp", (params, norm))
    assert st_t.ewald_used == 0 and st_m.ewald_used == 2
    for b in (0, g.nb - 1):
        assert np.array_equal(s_t.export_list(b), s_m.export_list(b))
    out = torch.empty((20000, NO), dtype=torch.float64, device="cuda")
    s_tr.ewald_points("exact", dev(offsets(name, 20000, 3)), out)
    cmax = np.abs(out.cpu().numpy()).max(0)
    mtot = (g.rho.reshape(g.nb, -1) * (1.0 / 2.0 ** (g.level - 1) / 8)[:, None] ** 3).sum()
    em, et = np.array(rep["err_mlp"]), np.array(rep["err_table"])
    r = taylor_reach()
    dphi = np.abs(pm - pt).max()
    da = np.abs(am - at).max()
    bphi = 2 * mtot * ((em[0] + 2 * et[0]) * cmax[0] + 3 * r * (em[1:4] * cmax[1:4]).max()) \
        + 1e-6 * np.abs(pt).max()
    ba = 2 * mtot * (((em[1:4] + 2 * et[1:4]) * cmax[1:4]).max() + 3 * r * (em[4:] * cmax[4:]).max()) \
        + 1e-6 * np.abs(at).max()
    print(f"{name} {grid}: |dPhi| {dphi:.3e} (bound {bphi:.3e}, max|Phi| {np.abs(pt).max():.3e}); "
          f"|da| {da:.3e} (bound {ba:.3e}, max|a| {np.abs(at).max():.3e}); "
          f"ms_eval table {st_t.ms_eval:.2f}, surrogate {st_m.ms_eval:.2f}")
    assert dphi <= bphi and da <= ba
    assert dphi <= 1e-4 * np.abs(pt).max() and da <= 1e-4 * np.abs(at).max()


@pytest.mark.parametrize("reach", [1.0, 3.0])
@pytest.mark.parametrize("name", list(BOXES))
def test_surrogate_walk_vs_oracle(trained, name, reach):
    """The device walk (network on FP16 matrix instructions, FP32 Taylor step
    and sums) against the oracle's FP64 walk with the same weights and the
    same grouping, cell by cell, on two sampled blocks of each of the deep
    grid's five levels (groups of 4^3, 2^3 and single cells).  Bound per cell:
    the per-pair FP16 bound of the network (forward_with_bound, its maximum
    over the folded domain and over the blocks' own offsets, doubled) summed
    over the list's masses, through the Taylor step (|delta| <= reach), plus
    the FP32 walk's rounding (1e-6 of max |Phi|, 1e-5 of max |a|).  With
    mlp_reach 3 the groups may reach three times the table's Taylor offset
    (4^3 groups already at h = 1/128)."""
    s_tr, _ = trained[name]
    params, norm = s_tr.mlp_get()
    bc, nroot = GRIDS[name]
    g = workloads.deep_amr(bc, nroot)
    rho = dev(g.rho.reshape(-1))
    (pm, am), st, s = solve32(g, rho, "mlp", (params, norm), mlp_reach=reach)
    # the same gravity when columns are on (the column walk leaves it to this walk)
    (pc, ac, _, _), _, _ = solve32(g, rho, "mlp", (params, norm), nside=1, mlp_reach=reach)
    assert np.array_equal(pc, pm) and np.array_equal(ac, am)
    rng = np.random.default_rng(31)
    sel = np.sort(np.concatenate([rng.choice(np.nonzero(g.level == lv)[0], 2, replace=False)
                                  for lv in range(3, 8)]))
    t = oracle.Tree(g, theta=0.5, ew_n=64, mlp_reach=reach)
    assert sorted({t.mlp_group_level(b) for b in sel}) == [0, 1, 2]
    if reach > 1:
        assert all(t.mlp_group_level(b) == 2 for b in sel if g.level[b] == 5)
    pr, ar, nint = t.walk_group_mlp(params, norm, sel)
    cells = (512 * sel[:, None] + np.arange(512)).ravel()
    # the per-pair bound: its maximum over random folded offsets and the
    # offsets from each sampled block's centre to its list's nodes
    ex = t.export()
    d = [offsets(name, 20000, 41)]
    for b in sel:
        cT = (np.asarray(g.coord[b]) + 0.5) / 2.0 ** (g.level[b] - 1)
        d.append(cT - ex["com"][t.block_list(b)])
    d = np.concatenate(d)
    L = np.asarray(g.nroot, float)
    d = np.where(np.asarray(g.bc, bool), d - L * np.floor(d / L + 0.5), d)
    d = d[np.abs(d[:, 2]) <= extent(name)[2]]
    _, bnd = forward_with_bound(params, norm, d)
    B = 2 * bnd.max(0)
    r = reach * taylor_reach()
    msum = np.array([ex["M"][t.block_list(b)].sum() for b in sel]).repeat(512)
    bphi = msum * (B[0] + 3 * r * B[1:4].max()) + 1e-6 * np.abs(pr).max()
    ba = msum * (B[1:4].max() + 3 * r * B[4:].max()) + 1e-5 * np.abs(ar).max()
    dphi = np.abs(pm[cells] - pr)
    da = np.abs(am[:, cells] - ar).max(0)
    print(f"{name}: surrogate walk vs oracle on {sel.size} blocks: max |dPhi| / bound {(dphi / bphi).max():.3f}, "
          f"max |da| / bound {(da / ba).max():.3f}; max |dPhi| / max|Phi| {dphi.max() / np.abs(pr).max():.2e}, "
          f"max |da| / max|a| {da.max() / np.abs(ar).max():.2e}; ms_eval {st.ms_eval:.2f}")
    assert (dphi <= bphi).all() and (da <= ba).all()
    assert st.n_interactions == 512 * (st.total_list - g.nb)


def test_walk_without_accepted_surrogate_is_the_table_walk():
    g = lognormal32((1, 1, 1))
    rho = dev(g.rho.reshape(-1))
    n = g.nb * 512
    outs = []
    for mode, accept in (("table", None), ("mlp", None), ("mlp", False)):
        s = ot.Solver.for_grid(g, theta=0.5, ewald_n=32, ewald=mode)
        if accept is not None:
            s.mlp_set(random_params(1), np.concatenate([extent("3p"), np.zeros(NO), np.ones(NO)]), accept=accept)
        s.build(rho)
        phi = torch.empty(n, dtype=torch.float32, device="cuda")
        acc = torch.empty(3 * n, dtype=torch.float32, device="cuda")
        st = s.solve(phi, acc)
        assert st.ewald_used == 0
        outs.append((phi.cpu(), acc.cpu()))
    for p, a in outs[1:]:
        assert torch.equal(p, outs[0][0]) and torch.equal(a, outs[0][1])


@pytest.mark.parametrize("name", list(BOXES))
def test_column_walk_with_surrogate(trained, name):
    """Columns (Nside 2) with the surrogate: the column walk computes the maps
    only and the surrogate walk the gravity.  Maps and tau are those of the
    table walk bit for bit; Phi and a those of the surrogate walk without
    columns bit for bit, within the accuracy budget of the table walk."""
    s_tr, rep = trained[name]
    params, norm = s_tr.mlp_get()
    nroot, _, bc = BOXES[name]
    g = lognormal32(bc, nroot)
    rho = dev(g.rho.reshape(-1))
    (pt, at, nt, tt), st_t, _ = solve32(g, rho, "table", nside=2)
    (pm, am, nm, tm), st_m, _ = solve32(g, rho, "mlp", (params, norm), nside=2)
    (pg, ag), _, _ = solve32(g, rho, "mlp", (params, norm))
    assert st_t.ewald_used == 0 and st_m.ewald_used == 2
    assert np.array_equal(nt, nm) and np.array_equal(tt, tm)
    assert np.array_equal(pg, pm) and np.array_equal(ag, am)
    dphi, da = np.abs(pm - pt).max(), np.abs(am - at).max()
    print(f"{name} columns: |dPhi| {dphi:.3e} (max|Phi| {np.abs(pt).max():.3e}), |da| {da:.3e} "
          f"(max|a| {np.abs(at).max():.3e}); ms_eval table {st_t.ms_eval:.2f}, surrogate {st_m.ms_eval:.2f}")
    assert dphi <= 1e-4 * np.abs(pt).max() and da <= 1e-4 * np.abs(at).max()


@pytest.mark.parametrize("name", list(BOXES))
def test_fused_column_walk_with_surrogate(trained, name):
    """192-pixel maps (in memory): one kernel carries the surrogate's gravity
    and the columns.  BH at theta = theta_pix = 0.25 gives the same lists with
    and without columns, so its Phi and a must equal the surrogate walk
    without columns (same network batches and Taylor step, the sums blocked
    per 60 instead of 64 entries: the FP32 walk's bars, 1e-6 of max |Phi|
    with its compensated sum and 1e-5 of max |a|) and its maps and tau the
    FP32 table column walk's bit for bit."""
    s_tr, _ = trained[name]
    params, norm = s_tr.mlp_get()
    bc, nroot = GRIDS[name]
    g = workloads.deep_amr(bc, nroot)
    rho = dev(g.rho.reshape(-1))
    kw = dict(theta=0.25)
    (pg, ag), st_g, s = solve32(g, rho, "mlp", (params, norm), **kw)
    (pf, af, nf, tf), st_f, sf = solve32(g, rho, "mlp", (params, norm), nside=4, **kw)
    (pt, at, nt, tt), st_t, _ = solve32(g, rho, "table", nside=4, **kw)
    assert st_f.ewald_used == 2 and st_f.total_list == st_g.total_list == st_t.total_list
    for b in (0, g.nb // 2, g.nb - 1):
        assert np.array_equal(s.export_list(b), sf.export_list(b))
    assert np.abs(pf - pg).max() <= 1e-6 * np.abs(pg).max()
    assert np.abs(af - ag).max() <= 1e-5 * np.abs(ag).max()
    assert np.array_equal(nf, nt) and np.array_equal(tf, tt)
    assert np.abs(pf - pt).max() <= 1e-4 * np.abs(pt).max() and np.abs(af - at).max() <= 1e-4 * np.abs(at).max()
    print(f"{name} fused 192-pixel walk: eval {st_f.ms_eval:.2f} ms (gravity walk {st_g.ms_eval:.2f} ms, "
          f"table column walk {st_t.ms_eval:.2f} ms)")


# --------------------------------------------- one list per 4^3 block octant
OCT_REACH = 6.0  # cell groups of 2^3 or 4^3 cells at every level of the deep grid


@pytest.mark.parametrize("name", list(BOXES))
def test_octant_lists_fused_walk_vs_oracle(trained, name):
    """list_group 4: the fused walk (surrogate gravity and 192-pixel maps)
    with one list per 4^3 octant of each block, against the oracle with the
    same octant lists, on two sampled blocks of each of the deep grid's five
    levels.  Lists bit-exact as sets (the device orders them level by level);
    Phi and a within the network's FP16 bound summed over each cell's own
    list masses plus the FP32 walk's rounding, as for the block lists; maps
    within 1e-5 of their maximum and tau within 1e-5 (the FP32 column walk's
    bars)."""
    s_tr, _ = trained[name]
    params, norm = s_tr.mlp_get()
    bc, nroot = GRIDS[name]
    g = workloads.deep_amr(bc, nroot)
    rho = dev(g.rho.reshape(-1))
    kw = dict(theta=0.25, mlp_reach=OCT_REACH)
    (pf, af, nf, tf), st, s = solve32(g, rho, "mlp", (params, norm), nside=4, list_group=4, **kw)
    assert st.ewald_used == 2
    assert st.n_interactions == 64 * (st.total_list - 8 * g.nb)
    rng = np.random.default_rng(37)
    sel = np.sort(np.concatenate([rng.choice(np.nonzero(g.level == lv)[0], 2, replace=False)
                                  for lv in range(3, 8)]))
    t = oracle.Tree(g, theta=0.25, ewald="table", ew_n=64, mlp_reach=OCT_REACH, list_group=4, nside=4)
    assert sorted({t.mlp_group_level(b) for b in sel}) == [1, 2]
    lists = {}
    for b in sel:
        for so in range(8):
            lists[b, so] = t.octant_list(b, so)
            got = np.sort(s.export_list(8 * b + so).astype(np.int64))
            assert np.array_equal(got, np.sort(lists[b, so])), (b, so)
    pr, ar, nint = t.walk_group_mlp(params, norm, sel)
    _, _, _, npr, tr = t.walk_group(sel, columns=True)
    cells = (512 * sel[:, None] + np.arange(512)).ravel()
    ex = t.export()
    d = [offsets(name, 20000, 43)]
    for b in sel:
        cT = (np.asarray(g.coord[b]) + 0.5) / 2.0 ** (g.level[b] - 1)
        d.append(cT - ex["com"][np.concatenate([lists[b, so] for so in range(8)])])
    d = np.concatenate(d)
    L = np.asarray(g.nroot, float)
    d = np.where(np.asarray(g.bc, bool), d - L * np.floor(d / L + 0.5), d)
    d = d[np.abs(d[:, 2]) <= extent(name)[2]]
    _, bnd = forward_with_bound(params, norm, d)
    B = 2 * bnd.max(0)
    r = OCT_REACH * taylor_reach()
    ci = np.arange(512)
    octs = ((ci % 8) // 4) + 2 * (((ci // 8) % 8) // 4) + 4 * ((ci // 64) // 4)
    msum = np.concatenate([np.array([ex["M"][lists[b, so]].sum() for so in range(8)])[octs] for b in sel])
    bphi = msum * (B[0] + 3 * r * B[1:4].max()) + 1e-6 * np.abs(pr).max()
    ba = msum * (B[1:4].max() + 3 * r * B[4:].max()) + 1e-5 * np.abs(ar).max()
    dphi = np.abs(pf[cells] - pr)
    da = np.abs(af[:, cells] - ar).max(0)
    nsel = nf.reshape(g.nb, 192, 512)[sel]
    dn = np.abs(nsel - npr).max() / np.abs(npr).max()
    dt = np.abs(tf[cells] - tr).max() / max(np.abs(tr).max(), 1.0)
    print(f"{name} octant lists: {st.total_list} entries over {8 * g.nb} lists; max |dPhi| / bound "
          f"{(dphi / bphi).max():.3f}, max |da| / bound {(da / ba).max():.3f}; maps {dn:.2e}, tau {dt:.2e}; "
          f"eval {st.ms_eval:.2f} ms")
    assert (dphi <= bphi).all() and (da <= ba).all()
    assert dn <= 1e-5 and dt <= 1e-5
    assert nint.sum() == sum(len(v) for v in lists.values())


def test_octant_lists_need_the_fused_walk(trained):
    """list_group 4 runs only in the fused walk: other solves of such a
    context and the adaptive update refuse it; list_group must be 0, 4 or 8."""
    s_tr, _ = trained["3p"]
    params, norm = s_tr.mlp_get()
    bc, nroot = GRIDS["3p"]
    g = workloads.deep_amr(bc, nroot)
    rho = dev(g.rho.reshape(-1))
    n = g.nb * 512
    cases = (("table", dict(nside=4, mlp_reach=OCT_REACH)),         # no surrogate
             ("mlp", dict(mlp_reach=OCT_REACH)),                     # no columns
             ("mlp", dict(nside=2, mlp_reach=OCT_REACH)),            # maps in LDS
             ("mlp", dict(nside=4)))                                 # single-cell groups at level 3
    for mode, kw in cases:
        with pytest.raises(ot.OTError) as e:
            solve32(g, rho, mode, (params, norm) if mode == "mlp" else None, list_group=4, **kw)
        assert e.value.status == ot.OT_ERR_UNSUPPORTED, (mode, kw)
    s = ot.Solver.for_grid(g, theta=0.5, ewald_n=64, ewald="mlp", nside=4, list_group=4, mlp_reach=OCT_REACH)
    s.mlp_set(params, norm, accept=True)
    s.build(rho)
    out = [torch.empty(k, dtype=torch.float64, device="cuda") for k in (n, 3 * n, 192 * n, n)]
    with pytest.raises(ot.OTError) as e:
        s.solve64(*out)
    assert e.value.status == ot.OT_ERR_UNSUPPORTED
    out = [o.float() for o in out]
    with pytest.raises(ot.OTError) as e:
        s.solve_abu(out[0], out[1], 1e-3, npix=out[2], tau=out[3], tol_tau=1e-3)
    assert e.value.status == ot.OT_ERR_UNSUPPORTED
    s.close()
    for bad in (2, 16):
        with pytest.raises(ot.OTError) as e:
            ot.Solver(bc=bc, list_group=bad)
        assert e.value.status == ot.OT_ERR_INVALID_ARG


def test_octant_lists_on_a_single_block(trained):
    """The degenerate grid: one 8^3 block filling a 3P box, mlp_reach 16 so
    that the 1/8 cells form 2^3 groups.  Every octant's list against the
    oracle's (as sets), Phi and a within 1e-4 of their maxima of the oracle's
    FP64 surrogate walk with the same lists and weights, maps 1e-5 and tau
    1e-5 of the oracle's walk."""
    s_tr, _ = trained["3p"]
    params, norm = s_tr.mlp_get()
    rho = np.random.default_rng(41).lognormal(0.0, 1.0, (1, 8, 8, 8))
    g = workloads.Grid((1, 1, 1), 1.0, (0.0, 0.0, 0.0), np.array([1], np.int32), np.zeros((1, 3), np.int32),
                       rho, (1, 1, 1), "one block")
    kw = dict(theta=0.25, mlp_reach=16.0)
    (pf, af, nf, tf), st, s = solve32(g, dev(g.rho.reshape(-1)), "mlp", (params, norm), nside=4, list_group=4,
                                      **kw)
    t = oracle.Tree(g, theta=0.25, ewald="table", ew_n=64, mlp_reach=16.0, list_group=4, nside=4)
    assert t.mlp_group_level(0) == 1
    for so in range(8):
        assert np.array_equal(np.sort(s.export_list(so).astype(np.int64)), np.sort(t.octant_list(0, so)))
    pm, am, _ = t.walk_group_mlp(params, norm, [0])
    _, _, _, npr, tr = t.walk_group([0], columns=True)
    assert np.abs(pf - pm).max() <= 1e-4 * np.abs(pm).max()
    assert np.abs(af - am).max() <= 1e-4 * np.sqrt((am ** 2).sum(0)).max()
    assert np.abs(nf.reshape(1, 192, 512) - npr).max() <= 1e-5 * np.abs(npr).max()
    assert np.abs(tf - tr).max() <= 1e-5 * max(np.abs(tr).max(), 1.0)
    assert st.total_list == sum(len(t.octant_list(0, so)) for so in range(8))
