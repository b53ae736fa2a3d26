"""Analytic velocity fields, evaluated pointwise.

Each constructor returns a callable f(x) -> u with x of shape [..., d] and u of
the same shape.  The callables accept numpy arrays or torch tensors (the math
module is picked from the argument), so large meshes can be sampled on the GPU.
Every field here has zero analytic divergence.
"""
import numpy as np


def _ns(x):
    try:
        import torch
        if torch.is_tensor(x):
            return torch
    except ImportError:  # pragma: no cover
        pass
    return np


def _stack(ns, comps):
    return ns.stack(comps, -1) if ns is np else ns.stack(comps, dim=-1)


def constant_field(c):
    c = np.asarray(c, dtype=np.float64)

    def f(x):
        ns = _ns(x)
        one = x[..., 0] * 0.0 + 1.0
        return _stack(ns, [one * float(ci) for ci in c])
    return f


def shear_field(coeffs_x, coeffs_z=None):
    """u = (p(y), 0, q(y)) (3D) or (p(y), 0) (2D) with polynomial p, q
    (coefficient lists, lowest degree first)."""
    def poly(c, y):
        out = y * 0.0
        for k, ck in enumerate(c):
            out = out + float(ck) * y ** k
        return out

    def f(x):
        ns = _ns(x)
        y = x[..., 1]
        comps = [poly(coeffs_x, y), y * 0.0]
        if x.shape[-1] == 3:
            comps.append(poly(coeffs_z or [0.0], y))
        return _stack(ns, comps)
    return f


def taylor_green_2d(freq=2.0 * np.pi):
    """(sin(w x) cos(w y), -cos(w x) sin(w y))."""
    def f(x):
        ns = _ns(x)
        a, b = freq * x[..., 0], freq * x[..., 1]
        return _stack(ns, [ns.sin(a) * ns.cos(b), -ns.cos(a) * ns.sin(b)])
    return f


def taylor_green_3d():
    """(sin x cos y cos z, -cos x sin y cos z, 0)."""
    def f(x):
        ns = _ns(x)
        a, b, c = x[..., 0], x[..., 1], x[..., 2]
        return _stack(ns, [ns.sin(a) * ns.cos(b) * ns.cos(c),
                           -ns.cos(a) * ns.sin(b) * ns.cos(c), a * 0.0])
    return f


def _half_space_modes(nmax, radius=None):
    modes = []
    r = range(-nmax, nmax + 1)
    for n in ((i, j, k) for i in r for j in r for k in r):
        if n == (0, 0, 0):
            continue
        first = next(v for v in n if v != 0)
        if first < 0:
            continue
        if radius is not None and (n[0] ** 2 + n[1] ** 2 + n[2] ** 2) > radius ** 2:
            continue
        modes.append(n)
    return np.array(modes, dtype=np.float64)


def curl_fourier_periodic(seed, nmax=4, scale=1.0):
    """u = curl A on the 2 pi-periodic cube,
    A = sum_{0<|n|<=nmax, half-space} a_n cos(n.x) + b_n sin(n.x), with
    a_n, b_n ~ N(0,1)^3; scaled so that the mean of |u|^2 over the period
    is scale^2 (closed form: RMS^2 = 1/2 sum |n x a_n|^2 + |n x b_n|^2)."""
    rng = np.random.default_rng(seed)
    kv = _half_space_modes(nmax, radius=nmax)
    a = rng.standard_normal(kv.shape)
    b = rng.standard_normal(kv.shape)
    ca = np.cross(kv, a)  # curl(a cos(n.x)) = -sin(n.x) (n x a)
    cb = np.cross(kv, b)  # curl(b sin(n.x)) =  cos(n.x) (n x b)
    rms = np.sqrt(0.5 * (np.sum(ca ** 2) + np.sum(cb ** 2)))
    ca *= scale / rms
    cb *= scale / rms
    return _fourier_sum(kv, -ca, cb)


def _fourier_sum(kv, sin_coef, cos_coef):
    """u(x) = sum_m sin(k_m.x) S_m + cos(k_m.x) C_m."""
    def f(x):
        ns = _ns(x)
        shp = x.shape[:-1]
        xf = x.reshape(-1, x.shape[-1])
        if ns is np:
            out = np.zeros_like(xf)
            K, S, C = kv, sin_coef, cos_coef
        else:
            out = ns.zeros_like(xf)
            K = ns.as_tensor(kv, dtype=xf.dtype, device=xf.device)
            S = ns.as_tensor(sin_coef, dtype=xf.dtype, device=xf.device)
            C = ns.as_tensor(cos_coef, dtype=xf.dtype, device=xf.device)
        chunk = 64
        for m0 in range(0, kv.shape[0], chunk):
            ph = xf @ K[m0:m0 + chunk].T
            out = out + ns.sin(ph) @ S[m0:m0 + chunk] + ns.cos(ph) @ C[m0:m0 + chunk]
        return out.reshape(shp + (x.shape[-1],))
    return f


def _fourier_sum6(kv, sin_coef, cos_coef):
    """Two three-component Fourier sums at once (coefficients [m][6]): one
    evaluation of each phase serves both.  On the GPU the modes go in chunks
    of up to 512 with the phase matrix held to 2^30 entries (it and its sine
    and cosine are the memory and the traffic), on the host in chunks of 64."""
    def f(x):
        ns = _ns(x)
        shp = x.shape[:-1]
        xf = x.reshape(-1, x.shape[-1])
        if ns is np:
            out = np.zeros((xf.shape[0], 6))
            K, S, C = kv, sin_coef, cos_coef
            chunk = 64
        else:
            out = ns.zeros((xf.shape[0], 6), dtype=xf.dtype, device=xf.device)
            K = ns.as_tensor(kv, dtype=xf.dtype, device=xf.device)
            S = ns.as_tensor(sin_coef, dtype=xf.dtype, device=xf.device)
            C = ns.as_tensor(cos_coef, dtype=xf.dtype, device=xf.device)
            chunk = max(16, min(512, (1 << 30) // max(xf.shape[0], 1)))
        for m0 in range(0, kv.shape[0], chunk):
            ph = xf @ K[m0:m0 + chunk].T
            out = out + ns.sin(ph) @ S[m0:m0 + chunk] + ns.cos(ph) @ C[m0:m0 + chunk]
        return out.reshape(shp + (6,))
    return f


def _curl_f_times_fourier(kv, a, b, fy, dfy):
    """u = curl(f(y) A), A = sum a_m cos(k.x) + b_m sin(k.x):
    u = f curl A + grad f x A, grad f = (0, f'(y), 0)."""
    ca = np.cross(kv, a)
    cb = np.cross(kv, b)
    # columns 0..2: curl A (sin: -n x a, cos: n x b); 3..5: A (sin: b, cos: a)
    both = _fourier_sum6(kv, np.concatenate([-ca, b], 1), np.concatenate([cb, a], 1))

    def f(x):
        ns = _ns(x)
        y = x[..., 1]
        cAA = both(x)
        cA, A = cAA[..., 0:3], cAA[..., 3:6]
        fp = dfy(y)
        gx = fp * A[..., 2]        # (0, f', 0) x A = (f' A_z, 0, -f' A_x)
        gz = -fp * A[..., 0]
        fv = fy(y)
        return _stack(ns, [fv * cA[..., 0] + gx, fv * cA[..., 1],
                           fv * cA[..., 2] + gz])
    return f


def field_rms(f, lengths, n=24):
    """Root mean square of |u| over a box by a tensor-product midpoint grid."""
    g = [(np.arange(n) + 0.5) / n * L for L in lengths]
    X = np.stack(np.meshgrid(*g, indexing="ij"), -1).reshape(-1, len(lengths))
    u = f(X)
    return float(np.sqrt(np.mean(np.sum(u ** 2, -1))))


def curl_fourier_wall(seed, nmax=4):
    """u = curl(f(y) A) on [0,1]^3, x and z periodic with period 1, walls at
    y = 0, 1; f = 16 y^2 (1-y)^2 (so u and its normal derivative of f vanish
    at the walls); A = sum_{0<|n|<=nmax, half-space} a_n cos(2 pi n.x) +
    b_n sin(2 pi n.x); scaled to RMS 1 by quadrature."""
    rng = np.random.default_rng(seed)
    nv = _half_space_modes(nmax, radius=nmax)
    kv = 2.0 * np.pi * nv
    a = rng.standard_normal(kv.shape)
    b = rng.standard_normal(kv.shape)
    fy = lambda y: 16.0 * y ** 2 * (1.0 - y) ** 2
    dfy = lambda y: 32.0 * y * (1.0 - y) * (1.0 - 2.0 * y)
    u0 = _curl_f_times_fourier(kv, a, b, fy, dfy)
    s = 1.0 / field_rms(u0, (1.0, 1.0, 1.0), n=20)
    return _curl_f_times_fourier(kv, a * s, b * s, fy, dfy)


def spectral_wall_field(seed, lengths=(4.0, 1.0, 2.0), nmax=8, slope=-17.0 / 6.0):
    """Turbulent-like field on [0,Lx]x[0,1]x[0,Lz], x and z periodic, walls at
    y = 0, 1: u = curl(f(y) A), wavevectors k = (2 pi n_x/Lx, 2 pi n_y,
    2 pi n_z/Lz), n in [-nmax, nmax]^3 minus 0 (half-space), |a_n|, |b_n|
    proportional to |k|^slope (|k|^(-17/6) gives E(k) ~ k^(-5/3)); RMS 1 by
    quadrature."""
    rng = np.random.default_rng(seed)
    r = range(-nmax, nmax + 1)
    nv = np.array([n for n in ((i, j, k) for i in r for j in r for k in r)
                   if n != (0, 0, 0) and next(v for v in n if v != 0) > 0],
                  dtype=np.float64)
    kv = 2.0 * np.pi * nv / np.array([lengths[0], 1.0, lengths[2]])
    amp = np.linalg.norm(kv, axis=1) ** slope
    a = rng.standard_normal(kv.shape) * amp[:, None]
    b = rng.standard_normal(kv.shape) * amp[:, None]
    fy = lambda y: 16.0 * y ** 2 * (1.0 - y) ** 2
    dfy = lambda y: 32.0 * y * (1.0 - y) * (1.0 - 2.0 * y)
    u0 = _curl_f_times_fourier(kv, a, b, fy, dfy)
    s = 1.0 / field_rms(u0, lengths, n=16)
    return _curl_f_times_fourier(kv, a * s, b * s, fy, dfy)
