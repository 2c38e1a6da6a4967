"""The continuous-batching server on the GPU: requests submitted while
others run are admitted into the running batch, and every result is the
same as the clip inpainted alone (bit-identical: batched kernels run the
same per-target arithmetic)."""
import time

import numpy as np
import pytest
import torch

from paper_1503_05528_amd import synth
from paper_1503_05528_amd.serve import GpuEngine, Request, Server

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone():
    from paper_1503_05528_amd import vi
    specs = [(synth.small(41 + i, 40 + 9 * i, 34 + 5 * i, 8 + i, levels=2, frac=0.04),
              dict(levels=2, seed=100 + i, em_tol=-1.0, em_max_iters=3)) for i in range(6)]
    ref = []
    for c, kw in specs:
        g = vi.Clip(torch.from_numpy(c.occluded_input()).cuda(), torch.from_numpy(c.mask).cuda(),
                    **kw)
        ref.append(g.inpaint().cpu().numpy())
        g.close()
    eng = GpuEngine(tune=(128, 2))
    srv = Server(eng, hbm_budget=4 << 30, max_slots=4)
    srv.start()
    futs = []
    for i, (c, kw) in enumerate(specs):
        futs.append(srv.submit(Request(c.occluded_input(), c.mask, kw,
                                       hole_fraction=float(c.mask.mean()))))
        time.sleep(0.01 * (i % 3))
    outs = [f.result(timeout=120) for f in futs]
    srv.stop()
    eng.close()
    for o, r in zip(outs, ref):
        assert np.array_equal(o, r)
    assert srv.max_running >= 2
    assert srv.latency_stats()["n"] == 6


def test_server_budget_queues_on_gpu():
    c = synth.small(50, 48, 40, 8, levels=2)
    kw = dict(levels=2, seed=1, em_tol=-1.0, em_max_iters=2)
    eng = GpuEngine(tune=(64, 2))
    need = eng.footprint(Request(c.occluded_input(), c.mask, kw))
    srv = Server(eng, hbm_budget=int(need * 1.5), max_slots=8)  # one at a time
    srv.start()
    futs = [srv.submit(Request(c.occluded_input(), c.mask, kw)) for _ in range(3)]
    outs = [f.result(timeout=120) for f in futs]
    srv.stop()
    eng.close()
    assert srv.max_running == 1
    assert all(np.array_equal(o, outs[0]) for o in outs)


def test_served_mean_results_equal_oracle():
    # plain-mean reconstructions are exact, so every served result equals
    # the oracle's inpainting of the same request bit for bit (Alg. 4)
    from oracle import vio
    print("[case] served MEAN results vs oracle", flush=True)
    specs = [(synth.small(141 + i, 40 + 11 * i, 34 + 6 * i, 8 + i, levels=2 + i % 2, frac=0.05),
              dict(levels=2 + i % 2, seed=400 + i, recon_mode=1)) for i in range(5)]
    eng = GpuEngine(tune=(128, 2))
    srv = Server(eng, hbm_budget=4 << 30, max_slots=3)
    srv.start()
    futs = []
    for i, (c, kw) in enumerate(specs):
        futs.append(srv.submit(Request(c.occluded_input(), c.mask, kw,
                                       hole_fraction=float(c.mask.mean()))))
        time.sleep(0.005 * (i % 2))
    outs = [f.result(timeout=120) for f in futs]
    srv.stop()
    eng.close()
    for i, (o, (c, kw)) in enumerate(zip(outs, specs)):
        ref = vio.Oracle(c.occluded_input(), c.mask, **kw).inpaint()
        assert np.array_equal(o, ref), i
