"""Seeded synthetic inputs shared by the GPU path and the oracle.

This module holds no lattice-Boltzmann arithmetic: it only draws the
initial density fields and the per-run parameters of the workloads, so
that both sides of every parity check receive byte-identical arrays.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014), used as a
counter-based generator: the value for (seed, stream, index) is

    u = splitmix64(splitmix64(seed ^ (stream * GOLDEN)) + index) >> 11
    u * 2**-53                      (a double in [0, 1))

so any single value can be regenerated without the others.

Initial profiles follow the paper's initialisations: the tanh droplet of
Eq. (24) and the tanh slab of Eq. (36) (here across x, with periodic
boundaries in both directions).
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 0x12044098
GOLDEN = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1


def _splitmix64_np(x: np.ndarray) -> np.ndarray:
    """Vectorised SplitMix64 finaliser applied to (x + GOLDEN)."""
    with np.errstate(over="ignore"):
        z = (x + np.uint64(GOLDEN)).astype(np.uint64)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix64(x: int) -> int:
    """Scalar SplitMix64 step (state increment by GOLDEN, then mix)."""
    z = (x + GOLDEN) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def uniform(seed: int, stream: int, index: np.ndarray | int) -> np.ndarray:
    """Counter-based uniform doubles in [0, 1) for (seed, stream, index)."""
    key = splitmix64((seed ^ ((stream * GOLDEN) & _M64)) & _M64)
    idx = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = _splitmix64_np(np.uint64(key) + idx)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def _noise(rho: np.ndarray, amp: float, seed: int, stream: int) -> np.ndarray:
    if amp == 0.0:
        return rho
    ny, nx = rho.shape
    u = uniform(seed, stream, np.arange(ny * nx, dtype=np.uint64)).reshape(ny, nx)
    return rho * (1.0 + amp * (2.0 * u - 1.0))


def slab(nx: int, ny: int, rho_l: float, rho_g: float, xa: float | None = None,
         xb: float | None = None, width: float = 2.0, noise: float = 0.0,
         seed: int = BASE_SEED, stream: int = 0) -> np.ndarray:
    """Liquid slab between x=xa and x=xb, tanh interfaces (Eq. 36 form).

    Returns rho0 as a C-contiguous float64 array of shape (ny, nx), row-major
    [y][x].  Multiplicative noise rho0 *= 1 + noise*(2u-1) per node.
    """
    xa = nx / 4.0 if xa is None else xa
    xb = 3.0 * nx / 4.0 if xb is None else xb
    x = np.arange(nx, dtype=np.float64)
    prof = rho_g + 0.5 * (rho_l - rho_g) * (np.tanh(2.0 * (x - xa) / width)
                                            - np.tanh(2.0 * (x - xb) / width))
    rho = np.broadcast_to(prof, (ny, nx)).copy()
    return np.ascontiguousarray(_noise(rho, noise, seed, stream))


def droplets(nx: int, ny: int, rho_l: float, rho_g: float, centers, radii,
             width: float = 2.0, noise: float = 0.0, seed: int = BASE_SEED,
             stream: int = 0) -> np.ndarray:
    """Circular liquid droplets with tanh profiles (Eq. 24 form).

    Distances are periodic (minimum image).  For several droplets the field is
    rho_g plus the sum of each droplet's excess over rho_g, which reduces to
    Eq. (24) exactly for a single droplet.
    """
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64),
                       np.arange(nx, dtype=np.float64), indexing="ij")
    rho = np.full((ny, nx), rho_g, dtype=np.float64)
    for (cx, cy), r0 in zip(centers, radii):
        dx = np.abs(x - cx)
        dx = np.minimum(dx, nx - dx)
        dy = np.abs(y - cy)
        dy = np.minimum(dy, ny - dy)
        r = np.sqrt(dx * dx + dy * dy)
        rho += 0.5 * (rho_l - rho_g) * (1.0 - np.tanh(2.0 * (r - r0) / width))
    return np.ascontiguousarray(_noise(rho, noise, seed, stream))


def droplet(nx: int, ny: int, rho_l: float, rho_g: float, r0: float,
            width: float = 2.0, noise: float = 0.0, seed: int = BASE_SEED,
            stream: int = 0) -> np.ndarray:
    """Single droplet of radius r0 centred at (nx/2, ny/2)."""
    return droplets(nx, ny, rho_l, rho_g, [(nx / 2.0, ny / 2.0)], [r0],
                    width, noise, seed, stream)


def droplet_layout(nx: int, ny: int, count: int, rmin: float, rmax: float,
                   gap: float = 16.0, seed: int = BASE_SEED, max_tries: int = 200000):
    """Seeded rejection sampling of non-overlapping droplets on a periodic box.

    Radius ~ U[rmin, rmax]; centres uniform; a candidate is kept when its
    periodic centre distance to every kept droplet is >= r_i + r_j + gap.
    Returns (centers, radii); raises if the box cannot hold them.
    """
    centers, radii = [], []
    k = 0
    while len(radii) < count:
        if k >= max_tries:
            raise RuntimeError("droplet_layout: could not place all droplets")
        u = uniform(seed, 7, np.arange(3 * k, 3 * k + 3, dtype=np.uint64))
        k += 1
        r = rmin + (rmax - rmin) * u[0]
        cx, cy = u[1] * nx, u[2] * ny
        ok = True
        for (ox, oy), orad in zip(centers, radii):
            dx = abs(cx - ox); dx = min(dx, nx - dx)
            dy = abs(cy - oy); dy = min(dy, ny - dy)
            if dx * dx + dy * dy < (r + orad + gap) ** 2:
                ok = False
                break
        if ok:
            centers.append((cx, cy))
            radii.append(r)
    return centers, radii


def sweep_runs(count: int, seed: int = BASE_SEED, lx=(64, 512, 32), ly=(16, 64, 16),
               t_range=(0.5, 0.95), tau_range=(0.6, 1.5), sigma_range=(0.0, 0.2)):
    """Per-run parameters of a batched flat-interface sweep.

    Lx uniform in {lx0, lx0+step, ..., lx1}, Ly likewise, T/Tc, tau and sigma
    uniform in their ranges.  Returns a list of dicts (one per run).
    """
    nlx = (lx[1] - lx[0]) // lx[2] + 1
    nly = (ly[1] - ly[0]) // ly[2] + 1
    runs = []
    for r in range(count):
        u = uniform(seed, 1000 + r, np.arange(5, dtype=np.uint64))
        runs.append(dict(
            nx=int(lx[0] + lx[2] * min(int(u[0] * nlx), nlx - 1)),
            ny=int(ly[0] + ly[2] * min(int(u[1] * nly), nly - 1)),
            t_over_tc=float(t_range[0] + (t_range[1] - t_range[0]) * u[2]),
            tau=float(tau_range[0] + (tau_range[1] - tau_range[0]) * u[3]),
            sigma=float(sigma_range[0] + (sigma_range[1] - sigma_range[0]) * u[4]),
        ))
    return runs


# --- sigma-surrogate network: seeded initial weights -------------------------

MLP_SHAPES = [("W1", (64, 3)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)),
              ("W3", (2, 64)), ("b3", (2,))]
MLP_NPARAMS = sum(int(np.prod(s)) for _, s in MLP_SHAPES)     # 4546


def mlp_init(seed: int = BASE_SEED) -> np.ndarray:
    """Initial parameters of the 3-64-64-2 network as one float32 vector.

    Weights ~ U(-1/sqrt(fan_in), +1/sqrt(fan_in)) from the counter-based
    generator, biases 0.  Layout: W1 (64x3, row = output unit), b1, W2 (64x64),
    b2, W3 (2x64), b3.
    """
    parts = []
    k = 0
    for name, shape in MLP_SHAPES:
        n = int(np.prod(shape))
        if name.startswith("W"):
            bound = 1.0 / np.sqrt(shape[1])
            u = uniform(seed, 5000, np.arange(k, k + n, dtype=np.uint64))
            parts.append(((2.0 * u - 1.0) * bound).astype(np.float32))
        else:
            parts.append(np.zeros(n, dtype=np.float32))
        k += n
    return np.concatenate(parts)
