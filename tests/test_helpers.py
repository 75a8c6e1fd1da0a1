"""The test-side check that explains a time-to-collision mismatch by a
near-threshold decision, pinned against the oracle's observation (no GPU)."""
import math

import numpy as np

from tests import helpers as H


def _two(O, p0, yaw0, v0, p1, yaw1, v1):
    prm = H.params()
    o = O.Oracle(H.world([(0, 0, 0, 300, 0), (0, 30, 0, 300, 30)]), prm)
    f, k = o.get_state()
    for n, (p, yaw, v) in enumerate(((p0, yaw0, v0), (p1, yaw1, v1))):
        f[0, n], f[1, n] = p
        f[3], f[6] = f[3], f[6]
        f[3, n], f[4, n], f[5, n], f[6, n] = math.cos(yaw / 2), 0, 0, math.sin(yaw / 2)
        f[7, n], f[8, n] = v
    f32 = f.astype(np.float32).astype(np.float64)
    o.set_state(f32, k)
    return o, f32, prm


def test_base_value_matches_the_oracle(oracle_mod):
    """On random pairs the helper's FP64 value is the oracle's TTC."""
    O = oracle_mod
    rng = np.random.default_rng(0)
    cr, cd = O.circle_model(H.params())
    hits = 0
    for _ in range(300):
        o, f, prm = _two(O, (0.0, 0.0), rng.uniform(-1, 1), tuple(rng.uniform(-10, 10, 2)),
                         tuple(rng.uniform(-25, 25, 2)), rng.uniform(-3, 3), tuple(rng.uniform(-10, 10, 2)))
        ttc = 10.0 * float(o.observe()[0, 206])
        ok, _ = H.ttc_explained(f, 0, 1, cr, cd, ttc, tol=1e-5)
        assert ok
        bad, _ = H.ttc_explained(f, 0, 1, cr, cd, ttc + 0.5 if ttc < 9 else ttc - 0.5, tol=1e-5)
        hits += ttc < 10.0
        # a value 0.5 s away is explained only by a near-threshold decision
        if bad:
            _, m = H.ttc_explained(f, 0, 1, cr, cd, ttc)
            assert m < H.TTC_MARGIN
    assert hits > 10


def test_abeam_neighbour_takes_either_branch(oracle_mod):
    """A neighbour exactly abeam and closing: the definition gives 10 s on
    the behind side and the swept-circle root on the other; both are
    explained, a third value is not."""
    O = oracle_mod
    cr, cd = O.circle_model(H.params())
    o, f, prm = _two(O, (0.0, 0.0), 0.0, (0.0, 0.0), (0.0, 8.0), 0.0, (0.0, -2.0))
    ttc = 10.0 * float(o.observe()[0, 206])
    root = (8.0 - 2 * cr) / 2.0
    assert abs(ttc - root) < 1e-6
    assert H.ttc_explained(f, 0, 1, cr, cd, root)[0]
    assert H.ttc_explained(f, 0, 1, cr, cd, 10.0)[0]
    assert not H.ttc_explained(f, 0, 1, cr, cd, 5.0)[0]
