"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke
check.

This module only draws inputs: workload parameters, nodal source values and
random vectors.  It holds none of the solver's arithmetic (no assembly, no
operator, no load-vector integration), so the CPU oracle and the GPU library
receive identical inputs without sharing any code path.

Workloads (names describe the problem; all use delta = 0, delta_hat = k,
Sommerfeld conditions on every face and V(2,2) scaled Jacobi, omega = 2/3):

  p1-64-k10        2D P1, 64 x 64 right-diagonal mesh, k = 10, 3 levels,
                   one Gaussian at (0.5, 0.5), sigma 0.05, complex FP64
  p1-1024-k100     2D P1, 1024 x 1024, k = 100, 8 levels, four Gaussians at
                   seeded uniform centres (PCG64 seed 0), sigma 0.02, FP64
  p1-2048-k200     2D P1, 2048 x 2048, k = 200, 9 levels (coarsest 8 x 8, as
                   for the 1024 mesh), Gaussian at (0.5, 0.5), sigma 0.05,
                   FP32 multigrid with FP64 outer iteration
  q1-256-k40       3D Q1, 256^3 hexahedra, k = 40, 6 levels, one Gaussian at a
                   seeded uniform centre (seed 0), sigma 0.03, FP32 multigrid
The paper's own sources (uniform f = 1 and the box source on
[0.4, 0.6]^2) are available for the paper-setting checks, with the paper's
meshes (PAPER_MESHES: c0 k^(3/2) cells per side, c0 = 1 rounded up to a
size the multigrid hierarchy divides) and its random initial guess
(paper_initial_guess).
"""

import numpy as np

WORKLOADS = {
    "p1-64-k10": dict(dim=2, n=64, k=10.0, delta=0.0, delta_hat=10.0, levels=3,
                      nrhs=1, precision="fp64", sigma=0.05, centres="centre"),
    "p1-1024-k100": dict(dim=2, n=1024, k=100.0, delta=0.0, delta_hat=100.0, levels=8,
                         nrhs=4, precision="fp64", sigma=0.02, centres="seed0"),
    "p1-2048-k200": dict(dim=2, n=2048, k=200.0, delta=0.0, delta_hat=200.0, levels=9,
                         nrhs=1, precision="fp32mg", sigma=0.05, centres="centre"),
    "q1-256-k40": dict(dim=3, n=256, k=40.0, delta=0.0, delta_hat=40.0, levels=6,
                       nrhs=1, precision="fp32mg", sigma=0.03, centres="seed0"),
}


def seeded_centres(count, dim, seed):
    """Source centres uniform on (0, 1)^dim from numpy's PCG64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.0, 1.0, size=(count, dim))


def workload_centres(name):
    w = WORKLOADS[name]
    if w["centres"] == "centre":
        return np.full((w["nrhs"], w["dim"]), 0.5)
    return seeded_centres(w["nrhs"], w["dim"], 0)


def node_coordinates(dim, n):
    """Nodal coordinates, lexicographic with x fastest, spacing 1/n."""
    t = np.arange(n + 1, dtype=np.float64) / n
    if dim == 2:
        y, x = np.meshgrid(t, t, indexing="ij")
        return [x.ravel(), y.ravel()]
    z, y, x = np.meshgrid(t, t, t, indexing="ij")
    return [x.ravel(), y.ravel(), z.ravel()]


def gaussian_nodal(dim, n, centre, sigma):
    """Nodal values of exp(-|x - centre|^2 / (2 sigma^2)), amplitude 1."""
    xs = node_coordinates(dim, n)
    r2 = sum((x - c) ** 2 for x, c in zip(xs, centre))
    return np.exp(-r2 / (2.0 * sigma * sigma))


def workload_sources(name, n=None):
    """Nodal Gaussian sources (nrhs, N) of a named workload (optionally on a
    different mesh size n, for reduced parity cases)."""
    w = WORKLOADS[name]
    nn = w["n"] if n is None else n
    return np.stack([gaussian_nodal(w["dim"], nn, c, w["sigma"])
                     for c in workload_centres(name)])


def uniform_source(dim, n):
    """The paper's uniform source f = 1 (nodal values)."""
    return np.ones((n + 1) ** dim)


def box_source(n, dim=2):
    """The paper's box source: 1 on [0.4, 0.6]^dim, 0 elsewhere (nodal)."""
    inside = np.ones((n + 1) ** dim, dtype=bool)
    for x in node_coordinates(dim, n):
        inside &= (x >= 0.4 - 1e-12) & (x <= 0.6 + 1e-12)
    return inside.astype(np.float64)


# k -> (cells per side, multigrid levels) for the paper's settings: the
# paper takes c0 k^(3/2) cells with c0 = 1 (64, 181, 512, 1448); sizes not
# divisible by 2^(levels-1) with a coarsest mesh of at most 4096 nodes are
# rounded up (c0 = 1.00, 1.02, 1.00, 1.02).
PAPER_MESHES = {16.0: (64, 3), 32.0: (184, 4), 64.0: (512, 5), 128.0: (1472, 7)}

# The meshes of the paper's weak-scaling runs (about 0.5 k^(3/2) cells per
# side in 2D, 0.54 k^(3/2) in 3D: 257^2 ... and 49^3, 129^3, 361^3 nodes),
# rounded to sizes the hierarchy divides down to a small coarsest mesh
# (c0 = 0.50, 0.49, 0.50, 0.49 in 2D): k -> (cells per side, levels).
WEAK_MESHES_2D = {64.0: (256, 6), 128.0: (704, 7), 256.0: (2048, 9), 512.0: (5632, 10),
                  1024.0: (16384, 12)}
WEAK_MESHES_3D = {20.0: (48, 3), 40.0: (128, 5), 80.0: (352, 6)}


def paper_initial_guess(count, seed):
    """The random initial guess of the paper's runs: real and imaginary
    parts uniform on [0, 1), as a PETSc random vector is drawn."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.random(count) + 1j * rng.random(count)


def random_complex(shape, seed):
    """Standard complex normal array (real and imaginary parts N(0, 1))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def serving_stream(count, sizes=(128, 256, 512, 1024), max_rhs=8, rate=None, seed=1,
                   coarsest=8):
    """Seeded request stream for the serving workload: mesh size n uniform
    over `sizes`, k = n/10, delta_hat = k, 1..max_rhs right-hand sides, each
    a Gaussian of sigma 2/n at a uniform centre, Poisson arrivals with the
    given rate (requests per second; None = all at t = 0).  Levels are chosen
    so the coarsest mesh has `coarsest` cells per side."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for i in range(count):
        n = int(rng.choice(np.asarray(sizes)))
        nrhs = int(rng.integers(1, max_rhs + 1))
        centres = rng.uniform(0.0, 1.0, size=(nrhs, 2))
        if rate:
            t += float(rng.exponential(1.0 / rate))
        levels = int(round(np.log2(n / coarsest))) + 1
        out.append(dict(id=i, n=n, k=n / 10.0, levels=levels, nrhs=nrhs, centres=centres,
                        sigma=2.0 / n, arrival=t))
    return out
