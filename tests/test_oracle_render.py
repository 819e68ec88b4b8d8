"""Closed-form and invariant pins of the oracle's compositing (Sec. 3,
Eq. 1-3), sampling and early termination (Sec. 6)."""
import numpy as np
import pytest
from scipy.special import expit

import oracle
import synth
from scene_builders import dense_scene

BYTES = [128, 200, 60, 128, 30, 250, 90, 170]       # per channel, constant everywhere


def deq(b, m):
    return 2.0 * m * b / 255.0 - m


def const_field(bytes_=BYTES):
    t = np.array([4 * deq(bytes_[c], 14 if c == 0 else 7) for c in range(8)])
    return np.exp(t[0]), expit(t[1:4]), expit(t[4:8])


def box_scene(lo, hi, bytes_=BYTES, L=64):
    """Constant bytes everywhere; occupancy = cells of the finest level (res L/4)
    whose box lies inside [lo, hi] (a box aligned to those cells)."""
    rf = L // 4
    h = 4.0 / rf
    c = -2.0 + (np.arange(rf) + 0.5) * h
    inx = (c >= lo[0]) & (c <= hi[0])
    iny = (c >= lo[1]) & (c <= hi[1])
    inz = (c >= lo[2]) & (c <= hi[2])
    occ = (inz[:, None, None] & iny[None, :, None] & inx[None, None, :]).astype(np.uint8)
    return dense_scene(L=L, R=L, fill_grid=lambda z, y, x, ch: np.asarray(bytes_)[ch] + 0 * x,
                       fill_planes=lambda pl, v, u, ch: np.asarray(bytes_)[ch] + 0 * u, occ_fine=occ)


def lattice(a, b, step):
    """Intervals of the uniform contracted lattice on segment a -> b: (midpoints, lengths)."""
    ell = np.linalg.norm(b - a)
    n = int(np.ceil(ell / step))
    u0 = np.arange(n) * step
    u1 = np.minimum(u0 + step, ell)
    um = 0.5 * (u0 + u1)
    e = (b - a) / ell
    return a + um[:, None] * e, u1 - u0, a + u0[:, None] * e, a + u1[:, None] * e


def in_box(p, lo, hi):
    return np.all((p >= lo) & (p < hi), axis=-1)


def mlp_np(scene, cd, F, d):
    W0, b0, W1, b1, W2, b2 = [a.astype(np.float64) for a in scene.mlp_split()]
    pe_s = np.concatenate([np.sin(d * 2.0 ** k) for k in range(4)])
    pe_c = np.concatenate([np.cos(d * 2.0 ** k) for k in range(4)])
    x = np.concatenate([cd, F, d, pe_s, pe_c])
    h = np.maximum(x @ W0 + b0, 0)
    h = np.maximum(h @ W1 + b1, 0)
    return h @ W2 + b2


def test_constant_density_box_inside_cube():
    lo, hi = np.array([0.0, -0.5, -0.5]), np.array([1.0, 0.5, 0.5])
    sc = box_scene(lo, hi)
    o = np.array([-0.3, 0.01, 0.02])
    d = np.array([1.0, 0.05, -0.03])
    d /= np.linalg.norm(d)
    out, st, log = oracle.render_ray(sc, o, d)
    # first segment: inside the cube, contracted == world; it ends on x = 1
    t_exit = (1.0 - o[0]) / d[0]
    mids, dl, _, _ = lattice(o, o + t_exit * d, sc.step)
    sel = in_box(mids, lo, hi)
    tot = dl[sel].sum()
    tau, cdiff, feat = const_field()
    T = np.exp(-tau * tot)
    assert st["evaluated"] == sel.sum()
    assert abs(st["T"] - T) < 1e-12
    assert abs(st["sum_w"] - (1 - T)) < 1e-12
    cd = (1 - T) * cdiff
    F = (1 - T) * feat
    assert np.allclose([st["cd0"], st["cd1"], st["cd2"]], cd, atol=1e-12)
    assert np.allclose([st["f0"], st["f1"], st["f2"], st["f3"]], F, atol=1e-12)
    assert np.allclose(out[:3], cd + mlp_np(sc, cd, F, d), atol=1e-12)
    assert abs(out[3] - (1 - T)) < 1e-12
    # world deltas equal contracted ones inside the unit cube
    out_w, st_w, _ = oracle.render_ray(sc, o, d, delta_mode=1)
    assert abs(st_w["T"] - T) < 1e-12


def test_step_to_zero_converges_to_chord():
    lo, hi = np.array([0.0, -0.5, -0.5]), np.array([1.0, 0.5, 0.5])
    sc = box_scene(lo, hi, bytes_=[130, 128, 128, 128, 128, 128, 128, 128])
    o = np.array([-0.3, 0.01, 0.02])
    d = np.array([1.0, 0.05, -0.03])
    d /= np.linalg.norm(d)
    tau = const_field([130, 128, 128, 128, 128, 128, 128, 128])[0]
    chord = 1.0 / d[0]                               # world length of x in [0, 1]
    for step in [1 / 16, 1 / 64, 1 / 256, 1 / 1024, 1 / 4096]:
        _, st, _ = oracle.render_ray(sc, o, d, step=step, t_min=0.0)
        opt = -np.log(st["T"]) / tau
        assert abs(opt - chord) <= step * (1 + 1e-9)


def test_constant_density_box_in_outer_region():
    # box in the +x outer slab of contracted space
    lo, hi = np.array([1.25, -0.5, -0.5]), np.array([1.75, 0.5, 0.5])
    sc = box_scene(lo, hi, bytes_=[100, 200, 60, 128, 30, 250, 90, 170])
    o = np.array([0.1, -0.05, 0.03])
    d = np.array([1.0, 0.2, -0.1])
    d /= np.linalg.norm(d)
    out, st, log = oracle.render_ray(sc, o, d, t_min=0.0)
    # Eq. 7 by hand: the ray leaves the cube on x = 1 and stays in region +x;
    # its contracted segment runs from the exit point to (2, d_y/d_x, d_z/d_x)
    t1 = (1.0 - o[0]) / d[0]
    a = o + t1 * d
    b = np.array([2.0, d[1] / d[0], d[2] / d[0]])
    mids, dl, y0, y1 = lattice(a, b, sc.step)
    sel = in_box(mids, lo, hi)
    tau = const_field([100, 200, 60, 128, 30, 250, 90, 170])[0]
    assert st["evaluated"] == sel.sum()
    assert abs(st["T"] - np.exp(-tau * dl[sel].sum())) < 1e-12
    # world deltas: the preimage of each contracted interval, from Eq. 7 by hand
    # (x_x = 1 / (2 - y_x), x_k = y_k x_x)
    def pre(y):
        ax = 1.0 / (2.0 - y[..., 0])
        return np.stack([ax, y[..., 1] * ax, y[..., 2] * ax], axis=-1)
    wl = np.linalg.norm(pre(y1[sel]) - pre(y0[sel]), axis=-1)
    _, st_w, _ = oracle.render_ray(sc, o, d, t_min=0.0, delta_mode=1)
    assert abs(st_w["T"] - np.exp(-tau * wl.sum())) < 1e-12 * max(1.0, np.exp(-tau * wl.sum()))


def test_early_termination_stops_marching():
    lo, hi = np.array([0.0, -0.5, -0.5]), np.array([1.0, 0.5, 0.5])
    sc = box_scene(lo, hi, bytes_=[230, 200, 60, 128, 30, 250, 90, 170])
    o = np.array([-0.3, 0.01, 0.02])
    d = np.array([1.0, 0.05, -0.03])
    d /= np.linalg.norm(d)
    out, st, log = oracle.render_ray(sc, o, d)
    ev = log[log["evaluated"] == 1]
    assert st["T"] < 2e-4
    # the last logged sample is the one that pushed T below the threshold
    assert log[-1]["evaluated"] == 1
    assert log[-1]["T"] * (1 - log[-1]["alpha"]) < 2e-4
    assert np.all(ev["T"][:-1] * (1 - ev["alpha"][:-1]) >= 2e-4)
    # without termination the march goes on
    _, st2, log2 = oracle.render_ray(sc, o, d, t_min=0.0)
    assert len(log2) > len(log)
    assert abs(st["sum_w"] + st["T"] - 1) < 1e-12


def test_weights_partition_unity_on_tiny(tiny_scene, tiny_cams):
    out, st = oracle.render(tiny_scene, tiny_cams)
    assert np.all(np.abs(st["sum_w"] + st["T"] - 1) < 1e-12)
    assert np.all(st["sum_w"] <= 1 + 1e-15)
    assert np.all((st["T"] >= 0) & (st["T"] <= 1))
    assert np.allclose(out[:, 3], 1 - st["T"])
    # colours and features are weighted means of sigmoids: within [0, sum_w]
    for f in ["cd0", "cd1", "cd2", "f0", "f1", "f2", "f3"]:
        assert np.all(st[f] >= 0) and np.all(st[f] <= st["sum_w"] + 1e-12)
    assert st["fragile"].mean() < 0.005
    assert st["evaluated"].sum() > 0


def test_empty_scene_gives_mlp_of_zero_features():
    sc = dense_scene(L=16, R=16, occ_fine=np.zeros((4, 4, 4), np.uint8))
    cams = synth.make_cameras([np.hstack([np.eye(3), np.zeros((3, 1))])], [(4, 3)])
    out, st = oracle.render(sc, cams)
    assert np.all(st["evaluated"] == 0)
    o, dirs = oracle.camera_rays(cams, 0, [0, 2], [0, 3])
    for k, (i, j) in enumerate([(0, 0), (2, 3)]):
        want = mlp_np(sc, np.zeros(3), np.zeros(4), dirs[k])
        assert np.allclose(out[i * 4 + j, :3], want, atol=1e-13)
    assert np.all(out[:, 3] == 0)


def test_camera_rays_pinhole():
    c2w = np.array([[0, 0, 1, 0.5], [1, 0, 0, -0.25], [0, 1, 0, 2.0]], float)   # z_cam -> +x world
    cams = synth.make_cameras([c2w], [(64, 48)], hfov_deg=90.0)
    o, d = oracle.camera_rays(cams, 0, [23, 0], [31, 63])
    assert np.allclose(o[0], [0.5, -0.25, 2.0])
    # pixel (23, 31) is half a pixel up-left of the principal point (32, 24)
    fx = 32.0
    v = np.array([-0.5 / fx, -0.5 / fx, 1.0])
    v /= np.linalg.norm(v)
    assert np.allclose(d[0], c2w[:, :3] @ v, atol=1e-7)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0)


def test_deterministic(tiny_scene, tiny_cams):
    a, _ = oracle.render(tiny_scene, tiny_cams, nthreads=1)
    b, _ = oracle.render(tiny_scene, tiny_cams, nthreads=4)
    assert np.array_equal(a, b)
