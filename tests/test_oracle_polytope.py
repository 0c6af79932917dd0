"""Pins of the oracle's general polytope corridor (Sec. III-D.1, P_i^H = {a_k . x <= b_k}), no GPU.

* an axis-aligned box written as its six faces gives the box iteration (a special
  case the box pins already fix);
* the iteration is equivariant under a rotation of space (waypoints and face
  normals rotated together), which a box corridor is not and which a wrong
  axis coupling in the polytope rows would break;
* on a tiny problem with tight faces the fixed point is the constrained optimum
  of an independent SQP solve.
"""
import copy

import numpy as np
import torch

from oracle import cadmm, references
from paper_2507_10290_amd.workloads import make_config, random_walk_batch


def _box_faces(lo, hi):
    F = np.zeros((lo.shape[0], 6, 4))
    for a in range(3):
        F[:, 2 * a, a] = 1.0
        F[:, 2 * a, 3] = hi[:, a]
        F[:, 2 * a + 1, a] = -1.0
        F[:, 2 * a + 1, 3] = -lo[:, a]
    return F


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_box_is_the_six_face_polytope():
    w = make_config(1, scale=12 / 1024)
    w.precision = "fp64"
    wp = copy.deepcopy(w)
    wp.faces = _box_faces(w.box_lo, w.box_hi)
    wp.box_lo = wp.box_hi = None
    r1 = cadmm.run(cadmm.problem_from_workload(w), 60)
    r2 = cadmm.run(cadmm.problem_from_workload(wp), 60)
    assert _rel(r2.c.numpy(), r1.c.numpy()) < 1e-12
    assert abs(r2.J.item() - r1.J.item()) < 1e-12 * r1.J.item()
    assert abs(r2.rp.item() - r1.rp.item()) < 1e-10 * r1.rp.item()


def test_rotating_space_rotates_the_iterates():
    w = random_walk_batch("rot", [5], [21], order=3, rho=1.0, precision="fp64", faces=8)
    P = w.waypoints
    for i in range(w.n_seg):                       # tight faces, so some become active
        for k in range(w.faces.shape[1]):
            a = w.faces[i, k, :3]
            w.faces[i, k, 3] = max(a @ P[i], a @ P[i + 1]) + 0.05
    R, _ = np.linalg.qr(np.random.Generator(np.random.PCG64(5)).standard_normal((3, 3)))
    wr = copy.deepcopy(w)
    wr.waypoints = w.waypoints @ R.T
    wr.faces = w.faces.copy()
    wr.faces[..., :3] = w.faces[..., :3] @ R.T
    pr, prr = cadmm.problem_from_workload(w), cadmm.problem_from_workload(wr)
    r1, r2 = cadmm.run(pr, 80), cadmm.run(prr, 80)
    c1 = cadmm.coeffs_by_axis(pr, r1.c).numpy()
    c2 = cadmm.coeffs_by_axis(prr, r2.c).numpy()
    assert _rel(c2, np.einsum("ab,sbn->san", R, c1)) < 1e-10
    assert abs(r2.J.item() - r1.J.item()) < 1e-10 * r1.J.item()
    # some face is active along the way (else the corridor would pin nothing)
    mats = cadmm.segment_matrices(pr)
    slack = mats["b"] - (mats["Ao"] @ r1.c[:, :, None])[..., 0]
    assert (slack < 0.05).any()


def _poly_active_problem():
    w = random_walk_batch("polypin", [3], [11], order=3, vmax=10.0, rho=100.0, precision="fp64",
                          dur=(1.5, 2.5), faces=8)
    P = w.waypoints
    for i in range(w.n_seg):
        for k in range(w.faces.shape[1]):
            a = w.faces[i, k, :3]
            w.faces[i, k, 3] = max(a @ P[i], a @ P[i + 1]) + 0.05
    L = np.linalg.norm(np.diff(P, axis=0), axis=1)
    w.vmax[:] = 1.875 * np.max(L / w.durations)   # the chord start is feasible
    return w


def test_polytope_fixed_point_matches_sqp():
    w = _poly_active_problem()
    pr = cadmm.problem_from_workload(w)
    c_ref, J_ref, res_sqp = references.constrained_reference(pr, tol=1e-12)
    assert res_sqp.status == 0, res_sqp.message
    res = cadmm.run(pr, 8000)
    c = cadmm.coeffs_by_axis(pr, res.c).numpy()
    assert abs(res.J.item() - J_ref[0]) / J_ref[0] < 1e-4
    assert np.linalg.norm(c - c_ref) / np.linalg.norm(c_ref) < 3e-3
    ck, Jk = references.kkt_reference(pr)
    assert J_ref[0] > Jk[0] * (1 + 1e-3)          # the faces are active at the optimum
