"""The whole hot-path step as the bench runs it (maps, grid-hopping decision,
its argmax seeding Block-OMP, direct decision and argmax, three Block-OMP
iterations, refinement) captured once in a HIP graph: three replays on new
frames, copied into the captured input buffer between replays, each equal bit
for bit to an eager step on the same frame.  The step is captured on one
stream, and on two: a second stream (default priority), forked from the
capture stream at the last selection and joined back into it, runs the last
Block-OMP fit and the direct decision and its argmax beside the refinement.
The eager path itself is checked against the FP64 oracle in test_gpu_parity.py.
"""
import numpy as np
import pytest
import torch

from paper_2307_16550_amd import gridhop as gh
from paper_2307_16550_amd import scene as sc

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("streams", [1, 2])
@pytest.mark.parametrize("cfg", [1, 2])
def test_step_graph_replays_match_eager(cfg, streams):
    dev = torch.device("cuda:0")
    s = sc.make_scene(cfg, 0)
    radar = gh.Radar.from_scene(s)
    grid = gh.grid_of(s.grid)
    dgrid_s = sc.direct_grid(s, cfg)
    dgrid = gh.grid_of(dgrid_s)
    y = torch.from_numpy(s.y).to(dev)
    dec = torch.empty(tuple(s.grid.n), dtype=torch.float32, device=dev)
    block = gh.peaks_tensor(s.grid.n[0] * s.grid.n[1], dev)
    arg = gh.peaks_tensor(1, dev)
    ws = torch.empty(gh.direct_workspace_bytes(radar, dgrid), dtype=torch.uint8, device=dev)
    ddec = torch.empty(tuple(dgrid_s.n), dtype=torch.float32, device=dev)
    dblock = gh.peaks_tensor(dgrid_s.n[0] * dgrid_s.n[1], dev)
    darg = gh.peaks_tensor(1, dev)
    bomp = gh.BompState(radar, grid, y, max_support=3)
    theta = torch.empty((3, 4), dtype=torch.float64, device=dev)
    rws = torch.empty(gh.refine_workspace_bytes(radar, grid, 3), dtype=torch.uint8, device=dev)

    maps = bomp.maps     # the frame's maps: the grid-hopping row's and Block-OMP's

    def step():
        gh.rd_maps(radar, y, maps)
        gh.decision(radar, grid, maps, gh.BILINEAR, dec=dec, block=block, want_argmax=False)
        bomp.reset()
        bomp.seed(block, selected=arg)
        gh.direct_decision(radar, dgrid, y, ws=ws, dec=ddec, block=dblock, want_argmax=False)
        gh.argmax(dblock, darg)
        bomp.fit()
        for _ in range(2):
            bomp.step()
        gh.refine(radar, grid, y, bomp.support, theta=theta, ws=rws)

    side = torch.cuda.Stream(device=dev)

    def step_two_streams():
        main_s = torch.cuda.current_stream()
        join = torch.cuda.Event()
        gh.rd_maps(radar, y, maps)
        gh.decision(radar, grid, maps, gh.BILINEAR, dec=dec, block=block, want_argmax=False)
        bomp.reset()
        bomp.seed(block, selected=arg)
        bomp.fit()
        bomp.step()
        bomp.select()
        selected = torch.cuda.Event()
        selected.record(main_s)
        side.wait_event(selected)
        with torch.cuda.stream(side):
            bomp.fit()
            gh.direct_decision(radar, dgrid, y, ws=ws, dec=ddec, block=dblock, want_argmax=False)
            gh.argmax(dblock, darg)
        gh.refine(radar, grid, y, bomp.support, theta=theta, ws=rws)
        join.record(side)
        main_s.wait_event(join)

    def outputs():
        return [t.clone() for t in (maps, dec, arg, ddec, darg, bomp.support, bomp.alpha, bomp.resid, theta)]

    step()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        if streams == 2:
            step_two_streams()
        else:
            step()
    for rep in range(3):
        s2 = sc.make_scene(cfg, 10 + rep)
        y.copy_(torch.from_numpy(s2.y).to(dev))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = outputs()
        step()
        torch.cuda.synchronize()
        want = outputs()
        names = ("maps", "dec", "arg", "ddec", "darg", "support", "alpha", "resid", "theta")
        for n, a, b in zip(names, got, want):
            assert torch.equal(a, b), f"replay {rep}: {n} differs from the eager step"
        print(f"cfg {cfg} streams {streams} replay {rep}: support {bomp.support.cpu().numpy()}", flush=True)
