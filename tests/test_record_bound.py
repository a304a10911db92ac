"""The force pass reads a particle's record cells only inside its ellipsoid
scaled about its centre by 1 + 1.5 / min(R_par, R_perp). Every fluid node
linked to the particle (a node n with n + c_i inside the ellipsoid, |c_i| <=
sqrt 2) must lie inside that region, or its record would be skipped. Checked
here on random ellipsoids, including thin disks and long needles."""
import numpy as np

LINKS = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1) if 0 < abs(a) + abs(b) + abs(c) <= 2]


def _rot(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _form(p, X, R, ra, rc):
    b = (p - X) @ R  # body frame: b = R^T (p - X)
    return (b[:, 0] ** 2 + b[:, 1] ** 2) / ra ** 2 + b[:, 2] ** 2 / rc ** 2


def test_linked_nodes_lie_in_scaled_ellipsoid():
    rng = np.random.default_rng(7)
    checked = 0
    for _ in range(120):
        rpar, rperp = rng.uniform(0.5, 9.0), rng.uniform(0.5, 9.0)
        if rng.random() < 0.3:  # extreme aspect ratios
            rperp = rpar * rng.choice([0.08, 12.0])
            rperp = min(rperp, 9.0)
        q = rng.normal(size=4)
        R = _rot(q / np.linalg.norm(q))
        X = rng.uniform(0.0, 1.0, 3)
        L = int(2 * max(rpar, rperp)) + 4
        g = np.stack(np.meshgrid(*[np.arange(-L, L + 1)] * 3, indexing="ij"), -1).reshape(-1, 3).astype(float)
        inside = g[_form(g, X, R, rperp, rpar) <= 1.0]
        s = 1.0 + 1.5 / min(rpar, rperp)
        for c in LINKS:
            n = inside - np.array(c, dtype=float)
            assert (_form(n, X, R, s * rperp, s * rpar) <= 1.0).all()
            checked += len(n)
    assert checked > 100000


def test_growing_each_axis_is_not_enough():
    """The plain alternative (every semi-axis grown by the link length) misses
    links near the tip of an elongated body, which is why the scaled form is
    used."""
    R = np.eye(3)
    X = np.zeros(3)
    rpar, rperp = 10.0, 0.6
    g = np.stack(np.meshgrid(*[np.arange(-14, 15)] * 3, indexing="ij"), -1).reshape(-1, 3).astype(float)
    inside = g[_form(g, X, R, rperp, rpar) <= 1.0]
    missed = 0
    for c in LINKS:
        n = inside - np.array(c, dtype=float)
        missed += int((_form(n, X, R, rperp + 1.5, rpar + 1.5) > 1.0).sum())
    assert missed > 0


def test_linked_nodes_clear_the_scaled_surface_by_a_margin():
    """The force pass evaluates the scaled-ellipsoid filter with reciprocals of
    the squared semi-axes instead of divisions, which moves the form by a few
    ulp. That is safe because linked nodes lie inside by far more: their form
    stays below ((1 + sqrt 2 / m) / (1 + 1.5 / m))^2, m = min(R)."""
    rng = np.random.default_rng(11)
    worst = 0.0
    for _ in range(60):
        rpar, rperp = rng.uniform(0.5, 9.0), rng.uniform(0.5, 9.0)
        q = rng.normal(size=4)
        R = _rot(q / np.linalg.norm(q))
        X = rng.uniform(0.0, 1.0, 3)
        L = int(2 * max(rpar, rperp)) + 4
        g = np.stack(np.meshgrid(*[np.arange(-L, L + 1)] * 3, indexing="ij"), -1).reshape(-1, 3).astype(float)
        inside = g[_form(g, X, R, rperp, rpar) <= 1.0]
        m = min(rpar, rperp)
        s = 1.0 + 1.5 / m
        bound = ((1.0 + np.sqrt(2.0) / m) / s) ** 2
        for c in LINKS:
            n = inside - np.array(c, dtype=float)
            f = _form(n, X, R, s * rperp, s * rpar)
            assert (f <= bound * (1 + 1e-12)).all()
            worst = max(worst, float(f.max()) if len(f) else 0.0)
    assert worst < 1.0 - 1e-4


def test_reciprocal_form_stays_within_the_raster_band():
    """The raster decides inside / outside with the division-free form unless
    it lies within 1e-9 of 1, and with the exact form (divisions) otherwise.
    The two forms must differ by far less than that band."""
    rng = np.random.default_rng(12)
    worst = 0.0
    for _ in range(40):
        rpar, rperp = rng.uniform(0.5, 40.0), rng.uniform(0.5, 40.0)
        q = rng.normal(size=4)
        R = _rot(q / np.linalg.norm(q))
        d = rng.uniform(-45.0, 45.0, (20000, 3))
        b = d @ R
        exact = (b[:, 0] * b[:, 0] + b[:, 1] * b[:, 1]) / (rperp * rperp) + (b[:, 2] * b[:, 2]) / (rpar * rpar)
        ia2, ic2 = 1.0 / (rperp * rperp), 1.0 / (rpar * rpar)
        fast = (b[:, 0] * b[:, 0] + b[:, 1] * b[:, 1]) * ia2 + (b[:, 2] * b[:, 2]) * ic2
        near = np.abs(exact - 1.0) < 0.5
        if near.any():
            worst = max(worst, float(np.abs(fast - exact)[near].max()))
        # decisions taken by the fast form outside the band agree with the exact form
        out = fast > 1.0 + 1e-9
        inn = fast < 1.0 - 1e-9
        assert (exact[out] > 1.0).all() and (exact[inn] <= 1.0).all()
    assert worst < 1e-13


def test_axis_aligned_box_holds_the_ellipsoid_and_is_tight():
    """The raster, shell and kill/fill passes walk the axis-aligned box of the
    rotated ellipsoid, with half extent sqrt(R_perp^2 (1 - o_k^2) + R_par^2 o_k^2)
    on axis k (o the body axis), and the force pass the same box of the
    ellipsoid scaled by 1 + 1.5 / min(R). Every lattice point inside the
    ellipsoid lies in the box, every linked node in the scaled box, and the box
    is attained: the surface point X + M e_k / sqrt(M_kk), M = R diag(R_perp^2,
    R_perp^2, R_par^2) R^T, lies on the ellipsoid at offset sqrt(M_kk) along k."""
    rng = np.random.default_rng(11)
    for _ in range(80):
        rpar, rperp = rng.uniform(0.5, 9.0), rng.uniform(0.5, 9.0)
        q = rng.normal(size=4)
        R = _rot(q / np.linalg.norm(q))
        X = rng.uniform(0.0, 1.0, 3)
        o = R[:, 2]
        e = np.sqrt(rperp ** 2 * (1.0 - o ** 2) + rpar ** 2 * o ** 2)
        L = int(2 * max(rpar, rperp)) + 4
        g = np.stack(np.meshgrid(*[np.arange(-L, L + 1)] * 3, indexing="ij"), -1).reshape(-1, 3).astype(float)
        inside = g[_form(g, X, R, rperp, rpar) <= 1.0]
        assert (np.abs(inside - X) <= e * (1.0 + 1e-9) + 1e-9).all()
        s = 1.0 + 1.5 / min(rpar, rperp)
        for c in LINKS:
            n = inside - np.array(c, dtype=float)
            assert (np.abs(n - X) <= s * e * (1.0 + 1e-9) + 1e-9).all()
        M = R @ np.diag([rperp ** 2, rperp ** 2, rpar ** 2]) @ R.T
        for k in range(3):
            p = X + M[:, k] / np.sqrt(M[k, k])
            assert abs(_form(p[None, :], X, R, rperp, rpar)[0] - 1.0) < 1e-12
            assert abs((p[k] - X[k]) - e[k]) < 1e-12 * max(rpar, rperp)
