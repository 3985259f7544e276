"""The traction-balance identity on the GPU (Eq. 4, Alg. 1, Alg. 2).

Quasi-static uniform compression of a flat pad on rollers by a plate that
covers the whole contact face: the exact solution is homogeneous, so sigma
takes the 1-D closed form (sigma_xx = sigma_yy = 0, sigma_zz from the lateral
stretch that zeroes sigma_xx), and the Alg. 1 traction integrated over the
contact face, sum_j t_j A_j, equals the negated indenter reaction of Alg. 2
(-sum_k f_k).  Run through the C ABI in both precisions."""
import numpy as np
import pytest
import scipy.optimize as so

from gpu_util import context, gpu_pad, log, voigt_to_mat
from oracle import contact, stepper
from workloads import scenes

pytestmark = pytest.mark.gpu
MM = 1e-3


def _rollers(X, Lx):
    fixed = np.zeros(X.shape[0], np.uint8)
    fixed[X[:, 2] == 0] = 4                                         # rollers: z fixed
    fixed[np.nonzero((X == 0).all(axis=1))[0]] = 7                  # pin origin
    fixed[np.nonzero((X[:, 0] == Lx) & (X[:, 1] == 0) & (X[:, 2] == 0))[0]] = 6
    return fixed


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("mixed", 1e-5)])
def test_uniform_compression_traction_balance(prec, tol):
    Lx, Ly, H = 18 * MM, 14 * MM, 4 * MM
    pad = scenes.box_pad(Lx, Ly, H, 6, 5, 2)
    X = pad.X
    fixed = _rollers(X, Lx)
    dhat, depth = 0.1 * MM, 0.2 * MM
    plate = scenes.Indenter(contact.BOX, (60 * MM, 60 * MM, 5 * MM, 0), np.eye(3),
                            np.array([Lx / 2, Ly / 2, H + dhat + 5 * MM - depth]))
    gp = gpu_pad(context(), pad, prec, fixed=fixed, quasi_static=1, dhat=dhat,
                 newton_tol=1e-12 if prec == "fp64" else 1e-9, cg_rel_tol=1e-10 if prec == "fp64" else 1e-5)
    st = gp.step([plate])
    assert st.status == 0
    x = gp.read("positions")
    op = stepper.make_pad(X, pad.tets, 0.3e6, 0.45, 1000.0, fixed=fixed)
    top = X[:, 2] == H
    s_z = x[top, 2].mean() / H
    mu, lam, a = op.mu[0], op.lam[0], op.alpha[0]
    s_x = so.brentq(lambda s: mu * s * s / (s * s * s_z) + lam * (s * s * s_z - a), 0.5, 1.5)
    J = s_x ** 2 * s_z
    szz = mu * s_z ** 2 / J + lam * (J - a)
    sig = voigt_to_mat(gp.read("sigma"))
    e_zz = np.abs(sig[:, 2, 2] - szz).max() / abs(szz)
    e_lat = max(np.abs(sig[:, 0, 0]).max(), np.abs(sig[:, 1, 1]).max()) / abs(szz)
    R = gp.read("reaction").ravel()
    ts = gp.read("traction_sum").ravel()
    f = gp.read("contact_force")
    bal = np.linalg.norm(ts + R) / np.linalg.norm(R)
    log(f"{prec}: {st} s_z {s_z:.6f} sigma_zz {szz:.4e} Pa, err zz {e_zz:.2e} lateral {e_lat:.2e}, "
        f"reaction {R}, traction sum {ts}, |sum t A + R| / |R| {bal:.2e}")
    assert np.ptp(x[top, 2]) < 1e-9 * H
    assert e_zz < tol and e_lat < tol
    assert bal <= 1e-3
    assert np.allclose(f.sum(axis=0), -R, rtol=1e-12, atol=1e-18)
    # compression: negative normal pressure on every contact-face triangle
    pn = gp.read("pressure").astype(np.float64)
    assert (pn[gp.read("surface_is_top").astype(bool)] < 0).all()
    gp.close()
