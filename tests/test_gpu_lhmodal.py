"""GPU parity of the free interface operator L_h in its modal form (the
cosine eigenbasis of the y-direction, exact for W = 0 on the uniform mesh)
against the FP64 oracle and against the dense-block form.

* L_h x on a problem with uneven strips, both Robin values and ny = 130
  (three 64-wide column tiles, ragged) and 20 traces (two 16-trace tiles,
  ragged): against the oracle's dense blocks, and against the GPU's dense
  form (lh_form).  The same at ny = 9, 65, 129 and 257, where ny - 1 is a
  power of two and the transforms run by FFT (lengths 16 to 512, with and
  without the radix-2 pass).
* The dense blocks formed from the modal form against the dense build.
* Full size (2048^2 cells, 64 uneven strips): L_h x on sampled strips
  against the oracle's free strip solve of that strip's inputs (the two
  outputs of strip j depend on its own inputs only).
* (I - L_h)^{-1} by GMRES in both forms.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle.schwarz import SchwarzOracle  # noqa: E402
from workloads import Problem  # noqa: E402

DEV = "cuda:0"


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _osm():
    from paper_1603_05110_amd import osm
    return osm


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def problem(ncy=129):
    cells = [5, 9, 7, 7, 12, 6, 8, 9, 5, 10, 7]
    return Problem(-4.0, 4.0, -3.0, 3.0, sum(cells), ncy, len(cells), cells, lap_coef=0.6,
                   beta=2.0, p=3.0, p_bc=1.5, dt=0.02)


def free_response(orc, j, x):
    """Outputs of strip j under L_h (traces 2(j-1) and 2j+1) from its inputs
    in x: the free strip problem with Robin data l_j, r_j, solved by the
    oracle's sparse LU (the definition the dense blocks are built from)."""
    pb, ny = orc.pb, orc.ny
    m = orc.mats[j]
    N = orc.N
    B = np.zeros((m.nx, ny), dtype=complex)
    My = m.My.toarray()
    if j >= 1:
        B[0] = -pb.lap_coef * (My @ x[2 * (j - 1) + 1])
    if j <= N - 2:
        B[-1] += -pb.lap_coef * (My @ x[2 * j])
    V = orc.free_solver(j).solve(B.ravel()).reshape(m.nx, ny)
    out = {}
    if j >= 1:
        out[2 * (j - 1)] = -2j * pb.p * V[0] - x[2 * (j - 1) + 1]
    if j <= N - 2:
        out[2 * j + 1] = -2j * pb.p * V[-1] - x[2 * j]
    return out


@pytest.mark.parametrize("ncy,form", [(129, "modal"), (8, "fft"), (64, "fft"), (128, "fft"),
                                      (256, "fft")])
def test_modal_lh_matvec_matches_oracle_and_dense_form(ncy, form):
    osm = _osm()
    pb = problem(ncy)
    log(f"modal L_h x: ny={pb.ncy + 1}, {pb.nsub} strips, expect {form}")
    orc = SchwarzOracle(pb, np.zeros((pb.ncx + 1, pb.ncy + 1)))
    orc.build_Lh()
    rng = np.random.default_rng(3)
    ntr = 2 * (pb.nsub - 1)
    x = rng.standard_normal((ntr, pb.ncy + 1)) + 1j * rng.standard_normal((ntr, pb.ncy + 1))
    want = orc.Lh_matvec(x.ravel()).reshape(x.shape)
    got = {}
    for dense in (False, True):
        s = osm.OsmSolver(pb, DEV, algo="precond", lh_form="dense" if dense else "modal")
        assert s.lh_form() == ("dense" if dense else form)
        got[dense] = s.interface_apply(osm.OSM_IFACE_LH, None, to_dev(x)).cpu().numpy()
        s.close()
    for dense in (False, True):
        assert rel(got[dense], want) < 1e-12, dense
        for t in range(ntr):
            assert rel(got[dense][t], want[t]) < 1e-12, (dense, t)
    assert np.max(np.abs(got[False] - got[True])) < 1e-12 * np.max(np.abs(want))
    # the free responses, strip by strip, pin the oracle's blocks too
    for j in (0, 4, pb.nsub - 1):
        for t, v in free_response(orc, j, x).items():
            assert rel(got[False][t], v) < 1e-12, (j, t)


@pytest.mark.parametrize("ncy", [70, 64])
def test_modal_dense_blocks_equal_the_dense_build(ncy):
    osm = _osm()
    pb = problem(ncy=ncy)
    blk = {}
    for dense in (False, True):
        s = osm.OsmSolver(pb, DEV, algo="precond", lh_form="dense" if dense else "modal")
        blk[dense] = s.get_lh_blocks().cpu().numpy()
        s.close()
    assert np.max(np.abs(blk[False] - blk[True])) < 1e-12 * np.max(np.abs(blk[True]))


@pytest.mark.parametrize("ncy", [99, 128])
def test_pinv_by_gmres_in_both_forms(ncy):
    """(I - L_h)^{-1} y by GMRES: (I - L_h) applied to the result gives y
    back (oracle's blocks), in the modal (dense transforms at ny = 100, FFT
    at ny = 129) and the dense form."""
    osm = _osm()
    pb = problem(ncy=ncy)
    orc = SchwarzOracle(pb, np.zeros((pb.ncx + 1, pb.ncy + 1)))
    orc.build_Lh()
    rng = np.random.default_rng(5)
    ntr = 2 * (pb.nsub - 1)
    y = rng.standard_normal((ntr, pb.ncy + 1)) + 1j * rng.standard_normal((ntr, pb.ncy + 1))
    for dense in (False, True):
        s = osm.OsmSolver(pb, DEV, algo="precond", lh_form="dense" if dense else "modal",
                          tol_gmres=1e-13, max_gmres=3000)
        x = s.interface_apply(osm.OSM_IFACE_PINV, None, to_dev(y)).cpu().numpy()
        s.close()
        back = x.ravel() - orc.Lh_matvec(x.ravel())
        assert rel(back, y.ravel()) < 1e-11, dense


def test_full_size_modal_lh_on_sampled_strips():
    """2048^2 cells, 64 uneven strips (ny = 2049: 33 column tiles, 126
    traces): L_h x on the first, a middle, the widest and the last strip
    against the oracle's free strip solves (the FFT of length 4096)."""
    from workloads import c5
    osm = _osm()
    pb = c5(steps=1).problems[0]
    log(f"full-size modal L_h: ny={pb.ncy + 1}, {pb.nsub} strips")
    rng = np.random.default_rng(7)
    ntr = 2 * (pb.nsub - 1)
    x = rng.standard_normal((ntr, pb.ncy + 1)) + 1j * rng.standard_normal((ntr, pb.ncy + 1))
    s = osm.OsmSolver(pb, DEV, algo="precond")      # ny = 2049: the modal form by default
    assert s.lh_form() == "fft"
    got = s.interface_apply(osm.OSM_IFACE_LH, None, to_dev(x)).cpu().numpy()
    s.close()
    orc = SchwarzOracle.__new__(SchwarzOracle)
    # only the strip matrices and Robin values are needed for free solves
    from oracle.fem import StripMatrices
    orc.pb, orc.N, orc.ny = pb, pb.nsub, pb.ncy + 1
    orc.cells = list(pb.strip_cells)
    orc.pl = [pb.p_bc if j == 0 else pb.p for j in range(pb.nsub)]
    orc.pr = [pb.p_bc if j == pb.nsub - 1 else pb.p for j in range(pb.nsub)]
    orc._free_lu = None
    cells = list(pb.strip_cells)
    sample = sorted({0, pb.nsub // 2, int(np.argmax(cells)), pb.nsub - 1})
    orc.mats = [StripMatrices(c, pb.ncy, pb.hx, pb.hy) if j in sample else None
                for j, c in enumerate(cells)]
    for j in sample:
        for t, v in free_response(orc, j, x).items():
            r = rel(got[t], v)
            log(f"  strip {j} ({cells[j]} cells) -> trace {t}: rel {r:.2e}")
            assert r < 1e-11, (j, t)
