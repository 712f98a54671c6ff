"""Pins of the FP64 material field F_m (oracle.c, "material neural field"):
hash-grid encoding after Mueller et al. (SIGGRAPH 2022, Sec. 3) with the
paper's configuration (Appendix A "Network details"), the 2-layer MLP, its
pull-back, and the field as the path tracer's material source (Sec. 3
"Intrinsic decomposition")."""
import copy
import math

import numpy as np
import pytest

from oracle.oracle import FieldRef, Oracle
from paper_2406_16360_amd import synth

LOGIT = lambda p: math.log(p / (1.0 - p))


def _field(levels=4, log2_table=10, n_min=4, n_max=64, seed=0, lo=(-1, -1, -1), hi=(1, 1, 1)):
    return synth.random_field(np.array(lo, np.float32), np.array(hi, np.float32), np.random.default_rng(seed),
                              levels=levels, log2_table=log2_table, n_min=n_min, n_max=n_max)


def _probe(f, feats, c=4.0):
    """A copy of f whose MLP passes features through: z1 = e + c (ReLU is the
    identity while |e| < c), outputs o = sigmoid(e[feats[o]])."""
    g = copy.deepcopy(f)
    I = 2 * f.levels
    g.w1 = np.zeros((32, I), np.float32)
    g.w1[np.arange(I), np.arange(I)] = 1.0
    g.b1 = np.full(32, c, np.float32)
    g.w2 = np.zeros((4, 32), np.float32)
    for o, i in enumerate(feats):
        g.w2[o, i] = 1.0
    g.b2 = np.full(4, -c, np.float32)
    return g


def _features(f, x):
    """All 2L encoded features at points x, read back through _probe."""
    I = 2 * f.levels
    out = np.zeros((len(x), I))
    for i0 in range(0, I, 4):
        feats = [min(i, I - 1) for i in range(i0, i0 + 4)]
        m = FieldRef(_probe(f, feats)).eval(x)
        e = np.log(m / (1.0 - m))
        for o, i in enumerate(feats):
            out[:, i] = e[:, o]
    return out


def test_level_resolutions_paper_config():
    """16 levels growing geometrically from N_min = 16 to N_max = 2048."""
    f = _field(levels=16, log2_table=12, n_min=16, n_max=2048)
    res = FieldRef(f).levels()
    assert res[0] == 16 and res[-1] == 2048 and len(res) == 16
    b = 128.0 ** (1.0 / 15.0)
    for l, n in enumerate(res):
        assert n <= 16 * b ** l + 1e-9 < n + 1
    assert np.all(np.diff(res) > 0)
    assert FieldRef(_field(levels=1, n_min=7, n_max=50)).levels().tolist() == [7]


def test_dense_levels_reproduce_affine_tables():
    """Levels whose (N+1)^3 vertices fit the table index them one-to-one
    (x fastest); trilinear interpolation of a table that is affine in the
    vertex coordinates reproduces that affine function of u N exactly."""
    f = _field(levels=2, log2_table=12, n_min=4, n_max=12)   # 5^3 and 13^3 <= 4096
    res = FieldRef(f).levels()
    coef = np.array([[0.11, -0.07, 0.05, 0.3], [-0.04, 0.09, 0.02, -0.2]])
    for l, N in enumerate(res):
        v = np.stack(np.meshgrid(*[np.arange(N + 1)] * 3, indexing="ij"), -1).reshape(-1, 3)
        slot = v[:, 0] + (N + 1) * (v[:, 1] + (N + 1) * v[:, 2])
        f.table[l] = 0.0
        for j in range(2):
            f.table[l, slot, j] = v @ coef[j, :3] / N + coef[j, 3]   # float32-rounded table
    x = np.random.default_rng(1).uniform(-1, 1, (200, 3))
    e = _features(f, x)
    u = (x + 1.0) / 2.0
    for l, N in enumerate(res):
        # what the float32 table holds at the cell corners, interpolated
        for j in range(2):
            exact = u @ coef[j, :3] + coef[j, 3]
            assert np.max(np.abs(e[:, 2 * l + j] - exact)) < 1e-6


def test_hashed_levels_partition_of_unity_and_axis_slots():
    """Hashed levels: the 8 trilinear weights sum to one (a constant table
    gives that constant); along the x axis the hash reduces to v0 mod T
    (first prime 1), so a grid vertex (v0, 0, 0) reads slot v0 mod T."""
    f = _field(levels=3, log2_table=8, n_min=40, n_max=300)   # every level hashed: 41^3 > 256
    f.table[:] = np.array([0.25, -0.5], np.float32)
    x = np.random.default_rng(2).uniform(-1, 1, (100, 3))
    e = _features(f, x)
    np.testing.assert_allclose(e[:, 0::2], 0.25, atol=1e-12)
    np.testing.assert_allclose(e[:, 1::2], -0.5, atol=1e-12)
    res = FieldRef(f).levels()
    T = f.table.shape[1]
    f.table[:] = np.random.default_rng(3).uniform(-1, 1, f.table.shape).astype(np.float32)
    for l, N in enumerate(res):
        v0 = np.array([0, 1, 7, N // 2, N - 1], np.int64)
        pts = np.stack([v0 / N * 2.0 - 1.0, -np.ones(5), -np.ones(5)], -1)
        e = _features(f, pts)
        np.testing.assert_allclose(e[:, 2 * l], f.table[l, v0 % T, 0], atol=1e-9)
        np.testing.assert_allclose(e[:, 2 * l + 1], f.table[l, v0 % T, 1], atol=1e-9)


def test_field_is_continuous_across_cells():
    """Trilinear interpolation is continuous: points just either side of a
    cell face at a hashed level give the same output (a swapped weight or a
    wrong corner offset breaks this)."""
    f = _field(levels=5, log2_table=9, n_min=16, n_max=200)
    ref = FieldRef(f)
    res = ref.levels()
    rng = np.random.default_rng(4)
    for N in res:
        base = rng.uniform(-0.9, 0.9, (20, 3))
        for a in range(3):
            k = np.floor((base[:, a] + 1.0) / 2.0 * N) + 1
            face = k / N * 2.0 - 1.0
            lo, hi = base.copy(), base.copy()
            lo[:, a] = face - 1e-10
            hi[:, a] = face + 1e-10
            assert np.max(np.abs(ref.eval(lo) - ref.eval(hi))) < 1e-7


def test_mlp_closed_forms():
    """W2 = 0: m = sigmoid(b2) everywhere.  W1 = 0: m = sigmoid(W2 relu(b1) + b2)."""
    f = _field()
    x = np.random.default_rng(5).uniform(-1, 1, (10, 3))
    g = copy.deepcopy(f)
    g.w2[:] = 0.0
    m = FieldRef(g).eval(x)
    np.testing.assert_allclose(m, np.tile(1.0 / (1.0 + np.exp(-g.b2.astype(np.float64))), (10, 1)), rtol=1e-14)
    g = copy.deepcopy(f)
    g.w1[:] = 0.0
    z2 = g.w2.astype(np.float64) @ np.maximum(g.b1.astype(np.float64), 0.0) + g.b2
    np.testing.assert_allclose(FieldRef(g).eval(x), np.tile(1.0 / (1.0 + np.exp(-z2)), (10, 1)), rtol=1e-14)


def test_field_outputs_clamp_domain():
    """Points outside [lo, hi] take the value at the nearest box point."""
    f = _field(lo=(0, 0, 0), hi=(2, 1, 4))
    ref = FieldRef(f)
    x = np.array([[-1.0, 0.5, 2.0], [3.0, 2.0, -7.0]])
    np.testing.assert_array_equal(ref.eval(x), ref.eval(np.clip(x, [0, 0, 0], [2, 1, 4])))


@pytest.mark.parametrize("which", ["table", "w1", "b1", "w2", "b2"])
def test_vjp_matches_central_differences(which):
    f = _field(levels=4, log2_table=9, n_min=8, n_max=90, seed=6)
    rng = np.random.default_rng(7)
    x = rng.uniform(-1, 1, (6, 3))
    g = rng.normal(size=(6, 4))
    vjp = FieldRef(f).vjp(x, g)[which]
    arr = getattr(f, which)
    if which == "table":   # entries the points actually touch
        idx = [tuple(i) for i in np.argwhere(np.abs(vjp) > 1e-6)]
        idx = [idx[i] for i in rng.choice(len(idx), 12, replace=False)]
    else:
        idx = [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(10)]
    for ix in idx:
        v0 = float(arr[ix])
        vals = []
        for s in (+1, -1):
            h = copy.deepcopy(f)
            getattr(h, which)[ix] = np.float32(v0 + s * 1e-3)
            vals.append((FieldRef(h).eval(x) * g).sum())
        dv = float(np.float32(v0 + 1e-3)) - float(np.float32(v0 - 1e-3))
        fd = (vals[0] - vals[1]) / dv
        assert abs(fd - vjp[ix]) <= 1e-5 * max(1.0, abs(fd)), (which, ix, fd, vjp[ix])


def _const_field(scene, m0):
    f = synth.random_field(scene.pos.min(0) - 0.1, scene.pos.max(0) + 0.1, np.random.default_rng(8),
                           levels=4, log2_table=10, n_min=4, n_max=40)
    f.w2[:] = 0.0
    f.b2 = np.array([LOGIT(v) for v in m0], np.float32)
    return f


def test_constant_field_renders_like_constant_vertex_materials():
    """A field whose output is the constant m0 renders exactly like per-vertex
    materials equal to (m0, metallic 0) everywhere, and its output-bias
    gradient is sigmoid'(b2) times the summed per-vertex gradient (the
    barycentric weights of a hit sum to one)."""
    w = synth.config1()
    m0 = (0.3, 0.55, 0.7, 0.4)
    f = _const_field(w.scene, m0)
    sc_f = synth.Scene(pos=w.scene.pos, faces=w.scene.faces, env=w.scene.env, mat_mode=synth.MAT_FIELD, field=f)
    mv = np.array([1.0 / (1.0 + math.exp(-float(b))) for b in f.b2] + [0.0], np.float32)
    sc_v = synth.Scene(pos=w.scene.pos, faces=w.scene.faces, env=w.scene.env, mat_mode=synth.MAT_VERTEX,
                       vmat=np.tile(mv, (w.scene.nv, 1)))
    items = synth.sample_items(w, 1500, 9)
    of, ov = Oracle(sc_f), Oracle(sc_v)
    rf, hf = of.render(w.views, w.opts, items)
    rv, hv = ov.render(w.views, w.opts, items)
    assert np.mean(hf == hv) > 0.999
    same = hf == hv
    np.testing.assert_allclose(rf[same], rv[same], rtol=1e-6, atol=1e-9)
    dl = np.random.default_rng(10).normal(size=(len(items), 3))
    for mode in (0, 1):
        opts = copy.deepcopy(w.opts)
        opts.grad_mode = mode
        gf = of.grad(w.views, opts, items[same], dl[same])
        gv = ov.grad(w.views, opts, items[same], dl[same])
        s = 1.0 / (1.0 + np.exp(-f.b2.astype(np.float64)))
        expect = s * (1.0 - s) * gv["vmat"][:, :4].sum(0)
        # (the vertex materials hold sigmoid(b2) rounded to float32)
        np.testing.assert_allclose(gf["b2"], expect, rtol=1e-5, atol=1e-6 * np.abs(expect).max())
        np.testing.assert_allclose(gf["env"], gv["env"], rtol=1e-5, atol=1e-6 * np.abs(gv["env"]).max())
        assert np.abs(gf["w2"]).sum() > 0      # the hidden activations see the gradient too


@pytest.mark.parametrize("which,grad_mode", [("table", 0), ("w1", 0), ("b1", 1), ("w2", 0)])
def test_path_gradient_matches_frozen_differences(which, grad_mode):
    """The field-parameter gradient of the frozen path functional against
    central differences of that functional (paths recorded once, field
    perturbed): pins the per-vertex seeding and the pull-back in the
    renderer."""
    w = synth.config1()
    # full-amplitude table: hidden units stay clear of the ReLU kink under the +-1e-3 steps
    sc = synth.with_field(w.scene, np.random.default_rng(11), levels=4, log2_table=10, n_min=4, n_max=60, decay=0.0)
    opts = copy.deepcopy(w.opts)
    opts.grad_mode = grad_mode
    o = Oracle(sc)
    items = synth.sample_items(w, 6, 12)
    rgb, _ = o.render(w.views, opts, items)
    dl = np.random.default_rng(13).normal(size=(len(items), 3))
    g = o.grad(w.views, opts, items, dl)[which]
    rng = np.random.default_rng(14)
    cand = np.argwhere(np.abs(g) > 1e-7)
    assert len(cand) > 0
    for ix in [tuple(cand[i]) for i in rng.choice(len(cand), min(5, len(cand)), replace=False)]:
        vals = []
        arr = getattr(sc.field, which)
        v0 = float(arr[ix])
        for s in (+1, -1):
            sc2 = copy.deepcopy(sc)
            getattr(sc2.field, which)[ix] = np.float32(v0 + s * 1e-3)
            o2 = Oracle(sc2)
            vals.append(sum(float(o.frozen(o2, w.views, opts, items[i]) @ dl[i]) for i in range(len(items))))
        dv = float(np.float32(v0 + 1e-3)) - float(np.float32(v0 - 1e-3))
        fd = (vals[0] - vals[1]) / dv
        assert abs(fd - g[ix]) <= 1e-5 * max(1.0, abs(fd)), (which, ix, fd, g[ix])
