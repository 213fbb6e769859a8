"""gh_refine_noalloc (the refinement with the library's static scratch) against
gh_refine on the same cells, through the C ABI: two calls in a row, the second
with fewer cells, so the second reuses the scratch the first left behind."""
import numpy as np
import pytest
import torch

from paper_2307_16550_amd import gridhop as gh
from paper_2307_16550_amd import scene as sc
from _fixtures import true_cell

POS_TOL = 1e-3     # m, the refinement bar
VEL_TOL = 1e-3     # m/s


def say(*a):
    print(*a, flush=True)


def starts_around(s, n_cells):
    """Each target's cell and its neighbours one step along each axis."""
    n = s.grid.n
    out = []
    for t in range(s.pos.shape[0]):
        idx0 = np.array(np.unravel_index(true_cell(s, t), n))
        out.append(int(np.ravel_multi_index(tuple(idx0), n)))
        for a in range(4):
            for d in (-1, 1):
                i = idx0.copy()
                i[a] += d
                if 0 <= i[a] < n[a]:
                    out.append(int(np.ravel_multi_index(tuple(i), n)))
    return out[:n_cells]


def refine_pair(gr, grid, y, cells):
    c = torch.tensor(cells, dtype=torch.int64, device="cuda:0")
    st_ref = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
    st_na = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
    ref = gh.refine(gr, grid, y, c, max_iter=100, status=st_ref)
    na = gh.refine_noalloc(gr, grid, y, c, max_iter=100, status=st_na)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), na.cpu().numpy(), int(st_ref.cpu()[0]), int(st_na.cpu()[0])


@pytest.mark.gpu
@pytest.mark.parametrize("cfg,first,second", [(2, 26, 3), (1, 9, 2)])
def test_refine_noalloc_matches_refine(cfg, first, second):
    s = sc.make_scene(cfg, 0)
    gr = gh.Radar.from_scene(s)
    grid = gh.grid_of(s.grid)
    y = torch.from_numpy(s.y).to("cuda:0")
    for n_cells in (first, second):
        cells = starts_around(s, n_cells)
        say(f"refine_noalloc cfg={cfg} cells={len(cells)}")
        ref, na, st_ref, st_na = refine_pair(gr, grid, y, cells)
        assert st_ref == 0 and st_na == 0
        assert np.all(np.isfinite(na))
        dp = float(np.max(np.abs(na[:, :2] - ref[:, :2])))
        dv = float(np.max(np.abs(na[:, 2:] - ref[:, 2:])))
        say(f"  |dpos| {dp:.3g} m, |dvel| {dv:.3g} m/s")
        assert dp <= POS_TOL and dv <= VEL_TOL
