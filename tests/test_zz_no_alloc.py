"""vi_onion_layer_noalloc (work buffers in the library's fixed device array)
against vi_onion_layer (work buffers allocated by the context): the same
layers, reconstructed values and shift maps bit for bit, for a clip and
then a smaller one, whose calls reuse the array the first clip's calls
left behind; a level beyond the array's limit is refused on the host."""
import numpy as np
import pytest
import torch

from paper_1503_05528_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vi():
    from paper_1503_05528_amd import vi as _vi
    _vi.lib()
    return _vi


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def peel(vi, clip, L, noalloc):
    g = vi.Clip(dev(clip.occluded_input()), dev(clip.mask), levels=L, seed=21)
    Hp = g.sets(L - 1)[0].clone()
    out = torch.empty((int(torch.count_nonzero(Hp)), 5), dtype=torch.float32, device="cuda")
    outs, hps = [], []
    layer = 0
    while True:
        o = g.onion_layer(Hp, layer, out=out, noalloc=noalloc)
        hps.append(host(Hp).copy())
        if len(o) == 0:
            break
        outs.append(host(o).copy())
        layer += 1
    state = [host(t).copy() for t in g.get_state(L - 1)]
    g.close()
    return outs, hps, state


def test_noalloc_layers_equal_allocating_layers(vi):
    cases = [(synth.small(91, 96, 72, 10, levels=2, frac=0.07), 2),
             (synth.small(92, 50, 40, 9, levels=2, frac=0.05), 2)]  # the second is smaller
    for i, (clip, L) in enumerate(cases):
        print(f"[case] no-alloc onion layers, clip {i} {clip.shape}", flush=True)
        a_out, a_hp, a_state = peel(vi, clip, L, noalloc=False)
        b_out, b_hp, b_state = peel(vi, clip, L, noalloc=True)
        assert len(a_out) == len(b_out) >= 2
        for x, y in zip(a_out, b_out):
            assert np.array_equal(x, y), i
        for x, y in zip(a_hp, b_hp):
            assert np.array_equal(x, y), i
        for x, y in zip(a_state, b_state):
            assert np.array_equal(x, y), i


def test_noalloc_refuses_a_level_beyond_its_array(vi):
    # 112 x 112 x 96 = 1 204 224 voxels at the coarsest (only) level, above
    # the 1 198 336 the fixed array holds: refused before any launch
    clip = synth.small(93, 112, 112, 96, levels=1, frac=0.01)
    g = vi.Clip(dev(clip.occluded_input()), dev(clip.mask), levels=1, seed=1)
    Hp = g.sets(0)[0].clone()
    with pytest.raises(vi.ViError) as e:
        g.onion_layer(Hp, 0, noalloc=True)
    assert e.value.status == -6
    assert torch.equal(Hp, g.sets(0)[0])
    g.close()
