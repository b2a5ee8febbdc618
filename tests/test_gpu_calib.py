"""The roofline calibration kernels (needs an MI355X): the copy reproduces its
source, and the atomic kernel adds exactly 64 x waves x instructions to the
target, in the line pattern its lanes-per-line setting states."""
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_calib_copy_exact():
    from paper_2109_13176_amd import gvom
    for n in (4, 4 * 1000 + 4, 1 << 22):  # int32 elements, multiples of 16 bytes
        src = torch.randint(-2**31, 2**31 - 1, (n,), dtype=torch.int32, device="cuda")
        dst = torch.zeros_like(src)
        assert gvom.map_calib_copy(dst, src) == 0
        torch.cuda.synchronize()
        assert torch.equal(dst, src)


@pytest.mark.parametrize("g", [1, 4, 16, 64])
def test_calib_atomic_counts(g):
    from paper_2109_13176_amd import gvom
    tgt = torch.zeros(1 << 16, dtype=torch.int32, device="cuda")
    n_waves, per_wave = 64, 8
    assert gvom.map_calib_atomic(tgt, n_waves, per_wave, g, seed=3) == 0
    torch.cuda.synchronize()
    assert int(tgt.sum()) == 64 * n_waves * per_wave
    lines = tgt.view(-1, 16)
    touched = lines[(lines != 0).any(1)]
    if g <= 16:
        # each group writes words 0, 16/g, 2*16/g, ... of its line
        step = 16 // g
        mask = torch.zeros(16, dtype=torch.bool, device="cuda")
        mask[::step] = True
        assert not bool((touched[:, ~mask] != 0).any())
    else:
        # four lanes on each word: every word of a touched line is a multiple of 4
        assert bool(((touched % 4) == 0).all()) and bool((touched > 0).all())


def test_calib_rejects_bad_arguments():
    from paper_2109_13176_amd import gvom
    tgt = torch.zeros(256, dtype=torch.int32, device="cuda")
    assert gvom.map_calib_atomic(tgt, 6, 1, 4) == gvom.MAP_E_INVALID   # waves not a multiple of 4
    assert gvom.map_calib_atomic(tgt, 4, 1, 3) == gvom.MAP_E_INVALID   # lanes per line
    a = torch.zeros(5, dtype=torch.int32, device="cuda")
    assert gvom.map_calib_copy(a, a.clone()) == gvom.MAP_E_INVALID     # 20 bytes
