"""Pin of the oracle's ray-mesh intersection (Eq. intersect; Appendix A
"Visibility estimation"): its BVH returns the plain minimum over all
triangles (ties to the lower primitive id) and the same any-hit answer."""
import numpy as np

from paper_2406_16360_amd import synth


def _rays(rng, n, radius=3.0):
    o = rng.normal(size=(n, 3))
    o = radius * o / np.linalg.norm(o, axis=1, keepdims=True)
    tgt = rng.normal(scale=0.6, size=(n, 3))
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    # a share of rays start on / inside the object
    inside = rng.random(n) < 0.3
    o[inside] = rng.normal(scale=0.5, size=(inside.sum(), 3))
    return o, d


def test_bvh_equals_bruteforce_c1(oracle_lib):
    w = synth.config1()
    o_ = oracle_lib.Oracle(w.scene)
    rng = np.random.default_rng(0)
    o, d = _rays(rng, 4000)
    p1, t1, a1, b1 = o_.trace(o, d)
    p2, t2, a2, b2 = o_.trace(o, d, brute=True)
    assert np.array_equal(p1, p2)
    hit = p1 >= 0
    assert hit.mean() > 0.3
    assert np.array_equal(t1[hit], t2[hit]) and np.array_equal(a1[hit], a2[hit])
    q1 = o_.trace(o, d, any_hit=True)[0]
    q2 = o_.trace(o, d, any_hit=True, brute=True)[0]
    assert np.array_equal(q1, q2)
    assert np.array_equal(q1 >= 0, hit)


def test_bvh_equals_bruteforce_displaced():
    from oracle import oracle as oo
    rng = np.random.default_rng(1)
    pos, faces, uv = synth.displaced_latlong_sphere(24, 48, 0.2, rng)
    sc = synth.Scene(pos=pos, faces=faces, env=np.ones((4, 8, 3), np.float32), mat_mode=0,
                     vmat=np.full((pos.shape[0], 5), 0.5, np.float32))
    o_ = oo.Oracle(sc)
    o, d = _rays(np.random.default_rng(2), 3000)
    p1, t1, _, _ = o_.trace(o, d)
    p2, t2, _, _ = o_.trace(o, d, brute=True)
    assert np.array_equal(p1, p2) and np.array_equal(t1[p1 >= 0], t2[p1 >= 0])


def test_edge_tie_and_degenerate(oracle_lib):
    # two coincident triangles: the lower id wins; a degenerate one never hits
    pos = np.array([[-1, -1, 0], [1, -1, 0], [0, 1, 0], [0, 0, 0], [1, 1, 0]], np.float32)
    faces = np.array([[0, 1, 2], [0, 1, 2], [3, 3, 4]], np.int32)
    sc = synth.Scene(pos=pos, faces=faces, env=np.ones((4, 8, 3), np.float32), mat_mode=0,
                     vmat=np.full((5, 5), 0.5, np.float32))
    o_ = oracle_lib.Oracle(sc)
    p, t, _, _ = o_.trace([[0, 0, 1.0]], [[0, 0, -1.0]])
    assert p[0] == 0 and t[0] == 1.0
    # a ray through the edge point shared by both is still a hit (inclusive)
    p, _, _, _ = o_.trace([[0, -1, 1.0]], [[0, 0, -1.0]])
    assert p[0] == 0
    # rays only ever hit at t > 0
    p, _, _, _ = o_.trace([[0, 0, -1.0]], [[0, 0, -1.0]])
    assert p[0] == -1
