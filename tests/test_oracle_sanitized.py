"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only).  The oracle's sources are built once more with the sanitizers
into a temporary directory, and a small workload runs through that build in
a child process with the sanitizer runtime preloaded: whole inpaintings
(MEAN and weighted, 1-3 levels, holes touching the volume border, temporal
subsampling, a 5x5x1 image), a teacher-forced search, the reduced patch
space's features, App. B's count and the realignment's motion estimate.
Any report ends the child with an error; its results must equal those of
the ordinary build."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRCS = [os.path.join(ROOT, "oracle", f) for f in ("vio.c", "vio_align.c", "vio_appb.c")]

WORKLOAD = r'''
import sys, numpy as np
sys.path.insert(0, ROOT)
from oracle import vio
from paper_1503_05528_amd import synth
out = {}
c = synth.small(23, 40, 34, 8, levels=2, frac=0.03)
c.mask[:] = 0
c.mask[0:3, 0:6, 0:7] = 1
c.mask[5:8, 28:34, 30:40] = 1
out["edge_mean"] = vio.Oracle(c.occluded_input(), c.mask, levels=2, seed=3, recon_mode=1,
                              em_max_iters=3, em_tol=-1.0).inpaint()
t = synth.tiny()
out["tiny_weighted"] = vio.Oracle(t.occluded_input(), t.mask, levels=1, seed=5,
                                  em_max_iters=3, em_tol=-1.0).inpaint()
s3 = synth.small(22, 50, 40, 20, levels=3, frac=0.04, kind="box")
out["temporal"] = vio.Oracle(s3.occluded_input(), s3.mask, levels=2, seed=2, recon_mode=1,
                             em_max_iters=2, em_tol=-1.0, temporal_subsample=1).inpaint()
im = synth.image(94, 64, 48, frac=0.05, levels=2)
out["image"] = vio.Oracle(im.occluded_input(), im.mask, levels=2, seed=7, recon_mode=1,
                          em_max_iters=2, em_tol=-1.0, patch=(5, 5, 1)).inpaint()
o = vio.Oracle(s3.occluded_input(), s3.mask, levels=2, seed=9)
rgbt, cand, dist, nvox = o.get_state(0)
o.nnf_search(0, 1)
out["search_cand"], out["search_dist"] = o.get_state(0)[1:3]
Q = o.pca_basis(0, 8, n_max=2048)
o.set_reduction(0, Q)
out["features"] = o.features(0, 8)
vol = synth.noise(4, (12, 14, 16))
ref = np.random.default_rng(1).integers(0, 256, (6, 3, 3, 3), dtype=np.uint8)
out["appb"] = vio.closer_than_constant(ref, vol, (3, 3, 3))
j, _ = synth.jittered(4, W=96, H=72, T=6)
out["align"] = vio.align_estimate(j.occluded_input(), j.mask)
np.savez(OUT, **out)
'''


def _run(env_extra, out_path):
    code = "ROOT = %r\nOUT = %r\n" % (ROOT, out_path) + WORKLOAD
    env = dict(os.environ, OMP_NUM_THREADS="2", **env_extra)
    return subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                          timeout=600)


@pytest.mark.timeout(900)
def test_oracle_clean_under_address_and_undefined_sanitizers(tmp_path):
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                             text=True).stdout.strip()
    if not os.path.isabs(libasan) or not os.path.exists(libasan):
        pytest.skip("no AddressSanitizer runtime for gcc")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-g", "-fPIC", "-shared", "-fopenmp",
                           "-ffp-contract=off", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           *SRCS, "-o", lib, "-lm"])
    ref = str(tmp_path / "ref.npz")
    r = _run({}, ref)
    assert r.returncode == 0, r.stderr[-3000:]
    san = str(tmp_path / "san.npz")
    r = _run({"VIO_LIB": lib, "LD_PRELOAD": libasan,
              "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
              "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}, san)
    report = r.stderr[-6000:]
    assert r.returncode == 0, report
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
    a, b = np.load(ref), np.load(san)
    assert sorted(a.files) == sorted(b.files)
    for k in a.files:
        assert np.array_equal(a[k], b[k]), k
