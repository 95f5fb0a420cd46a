"""The persisted tile cache through the library: a second lb_init of the same
configuration takes the pass and tile shapes from the cache file, picks the
same shapes, and gives bit-identical states."""
import numpy as np
import pytest

from paper_2101_04847_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2101_04847_amd import lb as mod
    return mod


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_cached_init_matches_timed_init(lb, storage, tmp_path, monkeypatch):
    import json
    path = tmp_path / "tiles.json"
    monkeypatch.setenv("LB_TILE_CACHE", str(path))
    st = {"f64": lb.F64, "f32": lb.F32}[storage]
    mem = []
    for seed, (nx, ny) in enumerate(((700, 300), (700, 300), (512, 200))):
        rA, rB = inputs.multi_mode(nx, ny, seed + 20)
        mem.append(lb.Member(nx, ny, rA, rB, tau=(1.0, 1.0), G=1.5, g=((0.0, -1e-4), (0.0, 1e-4))))
    print("[case] tile cache", storage, flush=True)
    a = lb.Lattice(mem, storage=st, poison=True)
    assert not a.tiles_cached
    rec = json.loads(path.read_text())
    assert len(rec) == 1
    (key, choice), = rec.items()
    assert key.startswith("gfx950") and "700x300,700x300,512x200" in key
    assert len(choice["th"]) == len(choice["th2"]) == len(choice["th3"]) == 2   # two size classes
    b = lb.Lattice(mem, storage=st, poison=True)
    assert b.tiles_cached
    assert b.steps_per_pass == a.steps_per_pass == choice["spp"]
    for m in range(3):
        assert b.tile_shape(m) == a.tile_shape(m)
    a.step(37)
    b.step(37)
    for m in range(3):
        assert np.array_equal(a.get_populations(m).cpu().numpy(), b.get_populations(m).cpu().numpy())
    a.close()
    b.close()
    # switched off: timed again, nothing recorded
    monkeypatch.setenv("LB_TILE_CACHE", "off")
    c = lb.Lattice(mem, storage=st)
    assert not c.tiles_cached
    c.close()
    assert json.loads(path.read_text()) == rec
