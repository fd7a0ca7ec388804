"""Seeded synthetic inputs shared by the tests, the benchmark and the serving loop.

This module holds workload parameters and random draws only -- none of the
method's arithmetic.  Everything the method computes from these parameters
(coordinates, reference atmosphere, initial perturbation, right-hand side) is
computed independently by the HIP library and by the CPU oracle.

The paper's own test cases (a rising thermal bubble in a box and a baroclinic
wave on the sphere, Sec. "Test Cases") are defined in publications that are
not restated here; the workloads below are synthetic stand-ins of the same
shape: hexahedral elements of low order on a box or a spherical shell, a
hydrostatic background plus a small potential-temperature perturbation.
"""
from __future__ import annotations

import numpy as np

# Physical constants of the dry atmosphere (J/(kg K), m/s^2, Pa).
PHYS = dict(R=287.0, cp=1004.5, g0=9.81, p0=1.0e5)

MESH_BOX = 0
MESH_SHELL = 1

IC_REST = 0
IC_BUBBLE = 1
IC_JET_BLOB = 2


def box_workload(nx, ny, nz, N, Lx, Ly, H, terrain=0.0, bubble_centre=None,
                 bubble_amp=0.5, bubble_radius=2000.0, noise_amp=1.0e-3, theta0=300.0,
                 periodic_z=False):
    """Mesh/physics/initial-condition parameters of a box workload (dict)."""
    if bubble_centre is None:
        bubble_centre = (Lx / 2.0, Ly / 2.0, 2000.0)
    return dict(
        mesh=dict(kind=MESH_BOX, N=N, ne=(nx, ny, nz), periodic=(1, 1, 1 if periodic_z else 0),
                  extent=(Lx, Ly, H), h0=terrain),
        phys=dict(PHYS, T0=theta0),
        ic=dict(kind=IC_BUBBLE, amp=bubble_amp, radius=bubble_radius, centre=tuple(bubble_centre),
                noise_amp=noise_amp),
    )


def small_box(N=4):
    """4x4x4 elements, 10 km cube, undeformed, periodic in x and y, N = 4;
    0.5 K cosine bubble of 2 km radius at (5, 5, 2) km, 1e-3 m/s velocity noise."""
    return box_workload(4, 4, 4, N, 10.0e3, 10.0e3, 10.0e3, terrain=0.0,
                        bubble_centre=(5.0e3, 5.0e3, 2.0e3))


def gpu_box(N=4):
    """One GPU's share: 64x64x16 elements on 400 x 400 x 20 km, terrain 500 m."""
    return box_workload(64, 64, 16, N, 400.0e3, 400.0e3, 20.0e3, terrain=500.0,
                        bubble_centre=(200.0e3, 200.0e3, 2.0e3))


def shell_workload(ne=32, nz=10, N=4, seed=0, a=6.371e6, H=30.0e3, T0=250.0):
    """Deep-atmosphere cubed-sphere shell: isothermal rest state, zonal jet
    20 m/s cos^2(lat), 1 K gaussian blob centred at a seeded (lon, lat)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lon = float(rng.uniform(0.0, 2.0 * np.pi))
    lat = float(rng.uniform(-np.pi / 3.0, np.pi / 3.0))
    return dict(
        mesh=dict(kind=MESH_SHELL, N=N, ne=(ne, ne, nz), periodic=(0, 0, 0), extent=(a, 0.0, H), h0=0.0),
        phys=dict(PHYS, T0=T0),
        ic=dict(kind=IC_JET_BLOB, amp=1.0, radius=500.0e3, centre=(lon, lat, 10.0e3), lz=3.0e3,
                jet_u0=20.0, noise_amp=0.0),
    )


def noise(n_unique: int, seed: int = 0) -> np.ndarray:
    """Standard normal draws [3][n_unique] (canonical unique order), PCG64(seed)."""
    return np.random.Generator(np.random.PCG64(seed)).standard_normal((3, n_unique))


def device_noise(n_unique: int, seed: int, device="cuda:0"):
    """Standard normal draws [3][n_unique] made on the device (torch's
    counter-based generator seeded with seed): the per-request noise of the
    serving workload, where the same request is compared with itself."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return torch.randn((3, n_unique), generator=g, device=device, dtype=torch.float64)


def random_state(n_unique: int, seed: int, rho_scale=1e-2, u_scale=1.0, theta_scale=0.5) -> np.ndarray:
    """Arbitrary nodal state [5][n_unique] (rho', u, v, w, theta') for parity
    checks that do not depend on a physical initial condition."""
    rng = np.random.Generator(np.random.PCG64(seed))
    q = np.empty((5, n_unique))
    q[0] = rho_scale * rng.uniform(-1.0, 1.0, n_unique)
    q[1:4] = u_scale * rng.standard_normal((3, n_unique))
    q[4] = theta_scale * rng.uniform(-1.0, 1.0, n_unique)
    return q


def serving_requests(n: int, seed: int, rate_per_s: float, orders=(3, 4, 5, 6),
                     meshes=((8, 8, 8), (16, 16, 16), (32, 32, 8), (64, 64, 16)), steps=50):
    """Poisson arrivals of ensemble-member requests: box mesh and order drawn
    uniformly, bubble position uniform in (x, y), z in [2 km, H - 2 km],
    amplitude in [0.1, 2] K, per-request noise seed.  Domain nx 6.25 km x
    ny 6.25 km x nz 1.25 km, terrain 500 m."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    reqs = []
    for r in range(n):
        t += float(rng.exponential(1.0 / rate_per_s))
        nx, ny, nz = meshes[int(rng.integers(len(meshes)))]
        N = int(orders[int(rng.integers(len(orders)))])
        Lx, Ly, H = nx * 6250.0, ny * 6250.0, nz * 1250.0
        centre = (float(rng.uniform(0, Lx)), float(rng.uniform(0, Ly)), float(rng.uniform(2000.0, H - 2000.0)))
        amp = float(rng.uniform(0.1, 2.0))
        wl = box_workload(nx, ny, nz, N, Lx, Ly, H, terrain=500.0, bubble_centre=centre, bubble_amp=amp)
        reqs.append(dict(id=r, arrival=t, workload=wl, noise_seed=int(rng.integers(1 << 31)), steps=steps))
    return reqs
