"""The Fig. 9-shaped tile kernel on the GPU: its four forms (every barrier,
two barriers eliminated, store/load promoted, tile in registers) give bitwise
equal results, and
those match the FP64 oracle within 6 u (u = 2^-24; positive inputs, one
rounded product and at most four tree additions per value)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2207_00257_amd import api, synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
U = 2.0 ** -24
FORMS = ("all", "eliminated", "promoted", "registers")


def run(form, h, v):
    hd = torch.from_numpy(np.ascontiguousarray(h)).to(DEV)
    vd = torch.from_numpy(v).to(DEV)
    out = torch.full((v.size,), np.nan, device=DEV)
    api.layerforward(hd, vd, out, form=form)
    torch.cuda.synchronize()
    return hd.cpu().numpy(), out.cpu().numpy()


@pytest.mark.parametrize("tiles", [1, 37, 1 << 16])
def test_forms_agree_and_match_oracle(tiles):
    rows = 16 * tiles
    h = synth.uniform_f32(rows * 16, 80 + tiles % 7).reshape(rows, 16)
    v = synth.uniform_f32(rows, 90 + tiles % 7)
    res = [run(f, h, v) for f in FORMS]
    for f, (nh, out) in zip(FORMS[1:], res[1:]):
        assert np.array_equal(nh.view(np.uint32), res[0][0].view(np.uint32)), f
        assert np.array_equal(out.view(np.uint32), res[0][1].view(np.uint32)), f
    ref_h, ref_o = oracle.layerforward(h, v)
    assert np.all(np.abs(res[0][0] - ref_h) <= 6 * U * ref_h)
    assert np.all(np.abs(res[0][1] - ref_o) <= 6 * U * ref_o)


def test_output_is_tile_row_zero():
    """Each tile's output equals its written-back row 0 (the column sums)."""
    h = synth.uniform_f32(16 * 16 * 5, 95).reshape(80, 16)
    v = synth.uniform_f32(80, 96)
    nh, out = run("eliminated", h, v)
    assert np.array_equal(out.reshape(5, 16), nh[0::16])
