"""The silver torus of the paper's plasmonics section (hole radius 20 nm, outer
radius 50 nm, so a 35 nm major and a 15 nm tube radius; silver from eq. 4.1):
the extinction peaks of the solved cross sections fall where the paper reports
its resonances, 342 and 530 nm for E along x and H along y (incidence normal to
the ring), and in addition 395 nm for E along x and H along z (needs an MI355X)."""

import numpy as np
import pytest

from synthetic import nystrom3, torus

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

UNIT = 10e-9                                   # length unit of the mesh: 10 nm
CASES = [("ExHy", [0.0, 0.0, 1.0], 342), ("ExHy", [0.0, 0.0, 1.0], 530), ("ExHz", [0.0, -1.0, 0.0], 395)]


@pytest.fixture(scope="module")
def ring():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return nystrom3(torus(3.5, 1.5, 72, 24))


def _cext(q, lam_nm, d):
    from paper_1211_7177_amd import materials, postprocess as pp
    from paper_1211_7177_amd.solver import BemProblem
    eps = complex(materials.silver_drude_lorentz(lam_nm * 1e-9))
    k0 = float(materials.wavenumber(lam_nm * 1e-9, UNIT))
    pb = BemProblem(q, k0, eps, order=12, order32=6)
    x, info = pb.solve(pb.rhs_planewave(d, [1.0, 0.0, 0.0]), tol=1e-5, restart=200, maxit=3000, mixed=True,
                       inner_tol=1e-2)
    cext = pp.cross_sections(pb, x, d, [1.0, 0.0, 0.0], k0, nt=16, nph=32)[0]
    pb.close()
    return cext


@pytest.mark.parametrize("name,d,paper_nm", CASES)
def test_extinction_peak_at_the_papers_resonance(ring, name, d, paper_nm):
    """C_ext on a 2 nm grid over paper +- 16 nm has an interior maximum within
    12 nm of the printed wavelength (mesh of 3456 triangles)."""
    lams = np.arange(paper_nm - 16, paper_nm + 17, 2)
    ce = np.array([_cext(ring, lam, d) for lam in lams])
    i = int(np.argmax(ce))
    print(name, paper_nm, "peak at", lams[i], "nm", " ".join("%d:%.4g" % (l, c) for l, c in zip(lams, ce)), flush=True)
    assert 0 < i < len(lams) - 1, "no interior maximum in the window"
    assert abs(lams[i] - paper_nm) <= 12
