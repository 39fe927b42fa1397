"""The optimiser's saved state (host side, no GPU): arrays and metadata
round-trip exactly, and a missing half reads as no state."""
import numpy as np

from paper_1903_07145_amd import optimize


def test_state_round_trip(tmp_path):
    rng = np.random.default_rng(0)
    st = dict(params=rng.random(107).astype(np.float32), m=rng.random(107).astype(np.float32),
              v=rng.random(107).astype(np.float32), guide_w=rng.random(50).astype(np.float32),
              guide_rec=rng.random((9, 16)).astype(np.float32), it=250, t=436.9,
              hist=dict(it=[0, 1], t=[0.1, 0.2], rmse=[0.3, 0.25], rmse_all=[0.4, 0.35], groups=[None, {"kd": 0.2}]),
              t_hit=None, t_hit_all=12.5)
    p = str(tmp_path / "state_x")
    optimize.save_state(p, st)
    back = optimize.load_state(p)
    for k in ("params", "m", "v", "guide_w", "guide_rec"):
        assert back[k].dtype == st[k].dtype and np.array_equal(back[k], st[k]), k
    assert back["it"] == 250 and back["t"] == 436.9 and back["t_hit"] is None and back["t_hit_all"] == 12.5
    assert back["hist"] == st["hist"]
    # a BRDF-arm state has no guide arrays
    st2 = dict(st, guide_w=None, guide_rec=None)
    optimize.save_state(p + "b", st2)
    b2 = optimize.load_state(p + "b")
    assert "guide_w" not in b2 and "guide_rec" not in b2


def test_missing_state(tmp_path):
    assert optimize.load_state(str(tmp_path / "none")) is None
    p = str(tmp_path / "half")
    open(p + ".json", "w").write("{}")
    assert optimize.load_state(p) is None
