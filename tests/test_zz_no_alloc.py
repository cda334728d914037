"""gks_conservation_sums_noalloc, the entry point that allocates nothing (its
partial sums live in a fixed device array of the library), against
gks_conservation_sums on the same contexts: two calls in a row through the
C-ABI, the second on a smaller mesh, to the 1e-12 normwise bar of the FP64
path (the two reduce in different orders), and bitwise equal when repeated."""
import ctypes

import numpy as np
import pytest

import paper_2102_01366_amd as G
from paper_2102_01366_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _sums_noalloc(s):
    out = torch.full((5,), float("nan"), dtype=torch.float64, device=s.device)
    st = s.L.gks_conservation_sums_noalloc(s._h, ctypes.c_void_p(out.data_ptr()))
    assert st == G.GKS_OK, s.L.gks_last_error(s._h)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_noalloc_sums_match_the_allocating_entry_point():
    big = I.kuhn_cube_mesh(24, 1.0, 0.1, 2, False)  # 82,944 cells, slip walls
    Wb, gWb = I.blast_cell_averages(big)
    small = I.kuhn_cube_mesh(5, 1.0, 0.1, 3, True)  # 750 cells: a ragged last block
    Ws, gWs = I.cell_averages(small, I.sine_wave_field())
    assert small.n_cell < big.n_cell
    for mesh, W, gW in ((big, Wb, gWb), (small, Ws, gWs)):
        s = G.Solver(mesh, G.default_config())
        s.init(W, gW)
        s.step_cfl(0.5)
        a = _sums_noalloc(s)
        b = s.conservation_sums()
        assert np.all(np.isfinite(a))
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max(), (a, b)
        np.testing.assert_array_equal(_sums_noalloc(s), a)


def test_noalloc_rejects_a_null_output():
    m = I.kuhn_cube_mesh(2, 1.0, 0.1, 4, True)
    W, gW = I.cell_averages(m, I.sine_wave_field())
    s = G.Solver(m, G.default_config())
    s.init(W, gW)
    assert s.L.gks_conservation_sums_noalloc(s._h, None) == G.GKS_E_INVAL
