"""Seeded liquid-fraction fields, right-hand sides and uncertainty samples.

The liquid fraction f_l in [0, 1] is the solver's masking input: cells with
f_l == 0 are fully solid (the paper's S tag, section 2.4) and drop out of the
pressure system; every other cell (liquid or mushy, tag LM) is solved.  The
fields here are synthetic stand-ins for the temperature-driven f_l of a real
solidification run.
"""
from __future__ import annotations

import numpy as np


def fl_linear_x(centres, x0=0.3, width=0.4):
    """f_l = clamp((x - x0) / width, 0, 1): solid for x <= x0."""
    return np.clip((centres[:, 0] - x0) / width, 0.0, 1.0)


def fl_planar_front(centres, seed=2, width=0.4, centre=(0.5, 0.5, 0.5), s_range=0.2):
    """Planar front with a seeded normal uniform on the sphere and offset
    s ~ U(-s_range, s_range): f_l = clamp((n.(x - centre) - s) / width, 0, 1)."""
    rng = np.random.default_rng(seed)
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    s = rng.uniform(-s_range, s_range)
    return np.clip(((centres - np.asarray(centre)) @ n - s) / width, 0.0, 1.0)


def fl_growing_front(centres, t, t_end, s_max=0.6, delta=0.1, axis=0, length=1.0):
    """Solid layer growing from the cold wall at x_axis = 0 as sqrt(t):
    s(t) = s_max * length * sqrt(t / t_end); f_l = clamp((x - s) / (delta*length), 0, 1)."""
    s = s_max * length * np.sqrt(max(t, 0.0) / t_end)
    return np.clip((centres[:, axis] - s) / (delta * length), 0.0, 1.0)


def rhs_uniform(n, seed=1, center_mask=None):
    """b ~ U(-1, 1) i.i.d. (PCG64 stream ``seed``); if ``center_mask`` is
    given, the mean over the masked entries is removed from those entries."""
    rng = np.random.default_rng(seed)
    b = rng.uniform(-1.0, 1.0, size=n)
    if center_mask is not None:
        m = np.asarray(center_mask, dtype=bool)
        if m.any():
            b[m] -= b[m].mean()
    return b


def batch_samples(n_samples=256, seed=3, param_seed=4, side_range=(24, 48)):
    """Uncertainty-quantification samples: cube side m ~ U{side_range}
    (inclusive), melt temperature ~ N(950, 10) K, mould wall temperature
    ~ N(600, 20) K, liquidus shift ~ U(-5, 5) K."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(side_range[0], side_range[1] + 1, size=n_samples)
    prng = np.random.default_rng(param_seed)
    t_melt = prng.normal(950.0, 10.0, size=n_samples)
    t_wall = prng.normal(600.0, 20.0, size=n_samples)
    d_liq = prng.uniform(-5.0, 5.0, size=n_samples)
    return [dict(side=int(sides[s]), t_melt=float(t_melt[s]), t_wall=float(t_wall[s]),
                 d_liq=float(d_liq[s])) for s in range(n_samples)]


def uq_front_fl(centres, sample, t, t_end, length=1.0, delta=0.1, t_liquidus=913.0):
    """Surrogate solid front of one uncertainty sample: a layer growing from
    the cold wall x = 0 as sqrt(t), its final depth set by how far the wall
    sits below the (shifted) liquidus relative to the melt superheat:
    s_max = 0.7 (T_liq + dT_liq - T_wall) / (T_melt - T_wall)."""
    t_liq = t_liquidus + sample["d_liq"]
    s_max = 0.7 * (t_liq - sample["t_wall"]) / (sample["t_melt"] - sample["t_wall"])
    return fl_growing_front(centres, t, t_end, s_max=s_max, delta=delta, axis=0, length=length)


def rhs_smooth_series(centres, t, seed=5, n_modes=6, noise=0.05, center_mask=None):
    """Right-hand side that changes smoothly in time, standing in for the
    velocity divergence of successive timesteps: a sum of n_modes products of
    low-order cosines, each with a seeded amplitude, frequency and phase in
    time, plus a small fixed noise field.  Centred over center_mask."""
    rng = np.random.default_rng(seed)
    x = np.asarray(centres)
    lo = x.min(axis=0)
    span = np.maximum(x.max(axis=0) - lo, 1e-30)
    u = (x - lo) / span
    b = np.zeros(x.shape[0])
    for _ in range(n_modes):
        k = rng.integers(0, 4, size=3)
        amp = rng.uniform(0.5, 1.5)
        omega = rng.uniform(5.0, 20.0)
        phase = rng.uniform(0, 2 * np.pi)
        b += amp * np.cos(omega * t + phase) * np.prod(np.cos(np.pi * k * u + rng.uniform(0, 1, 3)), axis=1)
    b += noise * rng.uniform(-1.0, 1.0, size=x.shape[0])
    if center_mask is not None:
        m = np.asarray(center_mask, dtype=bool)
        if m.any():
            b[m] -= b[m].mean()
    return b


def ustar_smooth_series(centres, t, seed=7, n_modes=6, scale=0.01, noise=0.05):
    """Intermediate velocity u* [n, 3] that changes smoothly in time (the
    predictor's output the pressure step corrects): per component, a sum of
    n_modes seeded products of low-order cosines with a time phase, times
    `scale`, plus a small fixed noise field."""
    rng = np.random.default_rng(seed)
    x = np.asarray(centres)
    lo = x.min(axis=0)
    span = np.maximum(x.max(axis=0) - lo, 1e-30)
    v = (x - lo) / span
    u = np.zeros((x.shape[0], 3))
    for d in range(3):
        for _ in range(n_modes):
            k = rng.integers(0, 4, size=3)
            amp = rng.uniform(0.5, 1.5)
            omega = rng.uniform(5.0, 20.0)
            phase = rng.uniform(0, 2 * np.pi)
            u[:, d] += amp * np.cos(omega * t + phase) * np.prod(
                np.cos(np.pi * k * v + rng.uniform(0, 1, 3)), axis=1)
    u += noise * rng.uniform(-1.0, 1.0, size=u.shape)
    return scale * u


def mlp_initial_weights(n_in=10, width=128, n_hidden=3, seed=0):
    """Initial weights of the warm-start network, drawn outside the method:
    for each layer (fan_out x fan_in), a row-major weight matrix followed by
    its bias, all U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from PCG64 stream seed,
    concatenated in layer order (the library's parameter layout)."""
    rng = np.random.default_rng(seed)
    dims = [n_in] + [width] * n_hidden + [1]
    parts = []
    for k in range(len(dims) - 1):
        fan_in, fan_out = dims[k], dims[k + 1]
        lim = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-lim, lim, size=fan_out * fan_in))
        parts.append(rng.uniform(-lim, lim, size=fan_out))
    return np.concatenate(parts)


def latin_hypercube(kinds, m, seed):
    """Latin-hypercube test points of the uncertainty wrapper: m points, one
    in each of the m equal-probability strata of every input (strata paired
    by independent seeded permutations), mapped to the standard input
    ("normal": standard normal, through the inverse distribution function;
    "uniform": on [-1, 1]).  Returns the points [m, d] and the underlying
    uniforms [m, d]."""
    from scipy.special import ndtri

    rng = np.random.default_rng(seed)
    d = len(kinds)
    U = np.empty((m, d))
    for j in range(d):
        U[:, j] = (rng.permutation(m) + rng.uniform(size=m)) / m
    X = np.empty_like(U)
    for j, kind in enumerate(kinds):
        X[:, j] = ndtri(U[:, j]) if kind == "normal" else 2.0 * U[:, j] - 1.0
    return X, U


def t_wall_layer(mesh, T_wall, T_melt, delta):
    """Temperature of a melt at T_melt that has cooled for a while against
    box walls held at T_wall: T = T_wall + (T_melt - T_wall) erf(d / delta),
    d the distance of the cell centre to the nearest face of the mesh's
    bounding box (a developed thermal boundary layer, so that a mushy zone
    and a solid rim exist from the first step)."""
    from scipy.special import erf

    x = mesh.nodes
    lo, hi = x.min(axis=0), x.max(axis=0)
    c = mesh.cell_centre
    d = np.minimum(c - lo, hi - c).min(axis=1)
    return T_wall + (T_melt - T_wall) * erf(d / delta)
