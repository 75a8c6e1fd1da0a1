"""The road-touch counters that give the roofline its road bytes, on cases
whose answer is known exactly (through the C ABI)."""
import numpy as np
import pytest

from paper_2605_08528_amd import inputs as I
from tests import helpers as H
from tests.helpers import params as mkparams

pytestmark = pytest.mark.gpu

SIZES = np.array([48, 4, 16, 4, 4, 9])


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a GPU"
    return T


def test_road_touch_counts_known_cases(torch):
    """One vehicle at rest at the centre of a flat square of two triangles
    split along the diagonal y = x (0.5 m triangle cells, a triangle listed
    in the cells it meets, within 1 mm): its four vertical wheel rays read
    one cell each.  The front-left wheel's cell [1.0, 1.5] x [0.5, 1.0] and
    the rear-right one's [-1.5, -1.0] x [-1.0, -0.5] touch the diagonal at a
    corner and hold both triangles, the other two cells one each, so the
    step reads 2 + 1 + 1 + 2 = 6 triangle records and 4 x 2 cell range
    entries, distinct per step.  With a road
    of polylines the observation reads exactly 64 distinct road points for
    its one agent, the occupancy of its cell once, and at least 64 point
    records.  Bytes are the item counts weighted by the item sizes; graph
    capture is refused while counting."""
    from paper_2605_08528_amd import sf
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        sim = sf.Sim(H.plain_worlds(1, 1), mkparams(), stream=stream)
        sim.road_touch(True)
        act = torch.zeros((1, 2), dtype=torch.float32, device="cuda")
        for _ in range(3):
            sim.step(act, 1.0 / 30.0, 4)
        items, nbytes, steps = sim.road_touch_read()
        assert steps == 3
        assert items[0].tolist() == [18, 24, 0, 0, 0, 0], items
        assert items[1].tolist() == [0] * 6, items
        assert nbytes.tolist() == (items * SIZES).sum(axis=1).tolist()
        sim.policy_load(*I.mlp_params([256, 256, 256, 2], seed=0))
        with pytest.raises(sf.SFError, match="road-touch"):
            sim.graph_capture(2, 1.0 / 30.0, 4)
        sim.road_touch(False)
        sim.graph_capture(2, 1.0 / 30.0, 4)
        sim.graph_launch()
        sim.close()

        w = I.intersections(1, 1, seed=4)
        sim = sf.Sim(w, mkparams(), stream=stream)
        sim.road_touch(True)
        sim.step(torch.zeros((1, 2), dtype=torch.float32, device="cuda"), 1.0 / 30.0, 4)
        items, nbytes, steps = sim.road_touch_read()
        print("one agent on an intersection:", items.tolist(), nbytes.tolist())
        assert steps == 1
        assert items[1, 5] == 64 and items[1, 4] == 1 and items[1, 2] >= 64 and items[1, 3] >= 2
        assert items[1, 0] == 0 and items[1, 1] == 0
        assert items[0, 2:].tolist() == [0, 0, 0, 0]
        assert items[0, 0] >= 4 and items[0, 1] >= 8
        torch.cuda.synchronize()
        sim.close()
