"""Seeded synthetic inputs shared by the HIP path, the oracle and the benchmark.

This module only generates inputs (phantom densities, source lists and the
parameter values of the synthetic material); it holds none of the transport
arithmetic.  Every generator is seeded, so both sides see identical inputs.

Workloads (units: cm, MeV, g/cm^3):
  water_pencil_32   1 MeV photon pencil on a 20 cm water cube, 32^3 voxels,
                    1e5 histories (FP64 parity case)
  hetero_broad_128  6 MeV 10x10 cm parallel photon field on a 25.6 cm cube,
                    128^3 voxels of 2 mm: water, a lung slab (rho 0.26) and 8
                    seeded bone spheres (rho 1.85), 1e7 histories
  electron_200      20 MeV electron pencil on a 20 cm water cube, 200^3 voxels
                    of 1 mm, 1e6 histories
  beamlets_256      512 photon beamlets (5x5 mm, 4-15 MeV, lognormal counts
                    summing to 5e7) on a 256^3 CT-like noise phantom
  hetero_broad_64   the heterogeneous phantom at 64^3 (4 mm), 6 MeV field,
                    1e7 histories (density-gradient case)
"""
from __future__ import annotations

import numpy as np

MC2 = 0.51099895000

# Synthetic "water": a single material whose cross sections are analytic
# models with these parameter values (see the material descriptor docs).
WATER = dict(
    z_mol=10.0,          # electrons per H2O molecule
    a_mol=18.01528,      # g/mol
    zz1_mol=76.0,        # 1*2 + 1*2 + 8*9
    z_screen=7.42,       # effective Z of the screening parameter
    i_exc=75.0e-6,       # MeV
    pe_coef=4.94, pe_eref=0.01, pe_exp=3.0,
    pp_coef=1.0e-3,
    ray_f0=10.0, ray_a=4.6,
    brems_b=0.016,
)

# Synthetic cortical-bone-like material (model parameters, not data): per
# formula unit 50 electrons and 96.2 g/mol (Z/A = 0.52), Z(Z+1) sum for an
# effective Z of 13.8, I = 106.4 eV; photoelectric, pair and bremsstrahlung
# coefficients raised with Z; Rayleigh F(0) = Z of the unit.
BONE = dict(
    z_mol=50.0, a_mol=96.2, zz1_mol=740.0, z_screen=13.8, i_exc=106.4e-6,
    pe_coef=28.5, pe_eref=0.01, pe_exp=3.0,
    pp_coef=1.9e-3,
    ray_f0=50.0, ray_a=4.6,
    brems_b=0.028,
)


# Synthetic lung-tissue-like material (model parameters, not data): per
# formula unit 10 electrons and 18.2 g/mol (Z/A = 0.549), Z(Z+1) sum for an
# effective Z of 7.6 (its small fractions of P, S, Cl, K raise it above
# water's), I = 75.3 eV; photoelectric coefficient raised by (7.6/7.42)^3,
# pair and bremsstrahlung coefficients by 7.6/7.42.
LUNG = dict(
    z_mol=10.0, a_mol=18.2, zz1_mol=80.0, z_screen=7.6, i_exc=75.3e-6,
    pe_coef=5.31, pe_eref=0.01, pe_exp=3.0,
    pp_coef=1.024e-3,
    ray_f0=10.0, ray_a=4.6,
    brems_b=0.0164,
)


def transport(e_max: float = 10.0, n_grid: int = 200, flags: int = 0, **kw) -> dict:
    t = dict(n_grid=n_grid, e_min=1.0e-3, e_max=e_max, eabs=(0.01, 0.1, 0.1),
             c1=0.05, c2=0.05, wcc=0.01, wcr=0.01, flags=flags)
    t.update(kw)
    return t


def water_cube(n: int, size: float, rho: float = 1.0) -> dict:
    d = size / n
    return dict(shape=(n, n, n), voxel=(d, d, d), origin=(0.0, 0.0, 0.0),
                rho=np.full((n, n, n), rho, dtype=np.float64))


def slab_phantom(nz: int, dz: float, rho_z, nxy: int = 1, dxy: float = 100.0) -> dict:
    """Laterally huge voxels, depth profile rho_z (length nz)."""
    rho = np.broadcast_to(np.asarray(rho_z, dtype=np.float64)[:, None, None], (nz, nxy, nxy)).copy()
    return dict(shape=(nz, nxy, nxy), voxel=(dxy, dxy, dz), origin=(0.0, 0.0, 0.0), rho=rho)


def block_phantom(n: int = 32, voxel=(0.4, 0.5, 0.6), seed: int = 6) -> dict:
    """Boxes of 1-6 voxels a side with densities drawn from {0.3, 1.0, 1.85},
    painted in random order over water, then 60 isolated voxels of density
    1.2: same-density regions of every size with ragged edges, on
    non-cubic voxels (x, y, z pitch 4, 5, 6 mm by default)."""
    rng = np.random.default_rng(seed)
    rho = np.ones((n, n, n))
    for _ in range(200):
        s = rng.integers(1, 7, size=3)
        o = rng.integers(0, n, size=3)
        rho[o[0]:o[0] + s[0], o[1]:o[1] + s[1], o[2]:o[2] + s[2]] = rng.choice([0.3, 1.0, 1.85])
    iso = rng.integers(0, n, size=(60, 3))
    rho[iso[:, 0], iso[:, 1], iso[:, 2]] = 1.2
    return dict(shape=(n, n, n), voxel=tuple(voxel), origin=(0.0, 0.0, 0.0), rho=rho)


def pencil(particle: int, energy: float, pos, n_hist: int, direction=(0.0, 0.0, 1.0)) -> dict:
    return dict(particle=particle, kind=0, energy=energy, pos=tuple(pos), dir=tuple(direction),
                width=(0.0, 0.0), n_hist=int(n_hist))


def rect_field(particle: int, energy: float, centre, width, n_hist: int) -> dict:
    return dict(particle=particle, kind=1, energy=energy, pos=tuple(centre), dir=(0.0, 0.0, 1.0),
                width=tuple(width), n_hist=int(n_hist))


def hetero_phantom(n: int, size: float = 25.6, seed: int = 2) -> dict:
    """Water background, lung slab rho 0.26 for z in [6, 12) cm over the full
    x-y extent, 8 bone spheres rho 1.85 with radius U(0.5, 1.5) cm and centres
    U([4, 21.6]^3) cm; a voxel belongs to a sphere if its centre does."""
    d = size / n
    c = (np.arange(n) + 0.5) * d
    rho = np.ones((n, n, n))
    z = c[:, None, None]
    rho[np.broadcast_to((z >= 6.0) & (z < 12.0), rho.shape)] = 0.26
    rng = np.random.Generator(np.random.PCG64(seed))
    radii = rng.uniform(0.5, 1.5, size=8)
    centres = rng.uniform(4.0, 21.6, size=(8, 3))
    zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
    for r, (cx, cy, cz) in zip(radii, centres):
        inside = (xx - cx) ** 2 + (yy - cy) ** 2 + (zz - cz) ** 2 <= r * r
        rho[inside] = 1.85
    return dict(shape=(n, n, n), voxel=(d, d, d), origin=(0.0, 0.0, 0.0), rho=rho)


def hetero_mm_phantom(n: int, size: float = 25.6, seed: int = 2) -> dict:
    """The heterogeneous phantom with materials: water (0) for the
    background, bone (1) for the spheres, lung (2) for the slab outside
    them."""
    ph = hetero_phantom(n, size, seed)
    mat = np.zeros(ph["rho"].shape, dtype=np.uint8)
    mat[ph["rho"] == 1.85] = 1
    mat[ph["rho"] == 0.26] = 2
    ph["mat"] = mat
    return ph


def ct_hu_volume(n: int = 32, seed: int = 7, sigma: float = 2.0) -> np.ndarray:
    """A CT-like volume of Hounsfield units (int16, [nz][ny][nx]): Gaussian-
    smoothed white noise mapped affinely to [-900, 1400] HU (lung to bone)."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.Generator(np.random.PCG64(seed))
    s = gaussian_filter(rng.standard_normal((n, n, n)), sigma)
    s = (s - s.min()) / (s.max() - s.min())
    return np.round(-900.0 + 2300.0 * s).astype(np.int16)


def ct_noise_phantom(n: int = 256, d: float = 0.2, seed: int = 3, sigma: float = 4.0) -> dict:
    """Gaussian-smoothed (sigma in voxels) white noise, affinely mapped to [0.2, 1.9]."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.Generator(np.random.PCG64(seed))
    noise = rng.standard_normal((n, n, n)).astype(np.float32)
    sm = gaussian_filter(noise, sigma=sigma, mode="wrap").astype(np.float64)
    lo, hi = sm.min(), sm.max()
    rho = 0.2 + (sm - lo) * (1.7 / (hi - lo))
    return dict(shape=(n, n, n), voxel=(d, d, d), origin=(0.0, 0.0, 0.0), rho=rho)


def beamlet_counts(nb: int = 512, total: int = 50_000_000, seed: int = 4, spread: float = 1.2,
                   lo: float = 1e3, hi: float = 1e6) -> np.ndarray:
    """n_b = clip(exp(m + spread z_b), lo, hi), m found by bisection so that the
    sum is `total`, then largest-remainder rounding to integers."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal(nb)

    def tot(m):
        return np.clip(np.exp(m + spread * z), lo, hi).sum()

    a, b = np.log(lo) - 10, np.log(hi) + 10
    for _ in range(200):
        m = 0.5 * (a + b)
        if tot(m) < total:
            a = m
        else:
            b = m
    x = np.clip(np.exp(0.5 * (a + b) + spread * z), lo, hi)
    x *= total / x.sum()
    base = np.floor(x).astype(np.int64)
    rem = int(total - base.sum())
    order = np.argsort(-(x - base), kind="stable")
    base[order[:rem]] += 1
    return base


def beamlet_sources(nb: int = 512, total: int = 50_000_000, size: float = 51.2, seed: int = 4):
    """512 beamlets of 5x5 mm on a 32 x 16 lattice at 5 mm pitch centred on the
    entrance face; energies U(4, 15) MeV (seed 4, drawn after the counts)."""
    counts = beamlet_counts(nb, total, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    energies = rng.uniform(4.0, 15.0, size=nb)
    nx, ny = 32, nb // 32
    srcs = []
    for b in range(nb):
        i, j = b % nx, b // nx
        cx = size / 2 + (i - (nx - 1) / 2) * 0.5
        cy = size / 2 + (j - (ny - 1) / 2) * 0.5
        srcs.append(rect_field(0, float(energies[b]), (cx, cy, 0.0), (0.5, 0.5), int(counts[b])))
    return srcs


def workload(name: str, n_hist: int | None = None) -> dict:
    """Named workload: phantom, sources, transport parameters, seed."""
    if name == "water_pencil_32":
        n = n_hist or 100_000
        return dict(name=name, phantom=water_cube(32, 20.0),
                    sources=[pencil(0, 1.0, (10.0, 10.0, 0.0), n)],
                    transport=transport(10.0, 200), seed=1, material=WATER)
    if name == "hetero_broad_128":
        n = n_hist or 10_000_000
        return dict(name=name, phantom=hetero_phantom(128),
                    sources=[rect_field(0, 6.0, (12.8, 12.8, 0.0), (10.0, 10.0), n)],
                    transport=transport(10.0, 200), seed=1, material=WATER)
    if name == "electron_200":
        n = n_hist or 1_000_000
        return dict(name=name, phantom=water_cube(200, 20.0),
                    sources=[pencil(1, 20.0, (10.0, 10.0, 0.0), n)],
                    transport=transport(100.0, 250), seed=1, material=WATER)
    if name == "beamlets_256":
        srcs = beamlet_sources(total=n_hist or 50_000_000)
        return dict(name=name, phantom=ct_noise_phantom(), sources=srcs,
                    transport=transport(100.0, 250), seed=1, material=WATER)
    if name == "hetero_broad_64":
        n = n_hist or 10_000_000
        return dict(name=name, phantom=hetero_phantom(64),
                    sources=[rect_field(0, 6.0, (12.8, 12.8, 0.0), (10.0, 10.0), n)],
                    transport=transport(10.0, 200), seed=1, material=WATER)
    if name in ("hetero_mm_64", "hetero_mm_128"):
        nn = 64 if name.endswith("64") else 128
        n = n_hist or 10_000_000
        return dict(name=name, phantom=hetero_mm_phantom(nn),
                    sources=[rect_field(0, 6.0, (12.8, 12.8, 0.0), (10.0, 10.0), n)],
                    transport=transport(10.0, 200), seed=1, material=WATER, materials=[WATER, BONE, LUNG])
    if name == "target_detector":
        # 2 MeV electrons stopped in a 1.5 cm water target, a 10 cm air gap,
        # a 2 cm water detector that only bremsstrahlung photons reach
        # (layers of 0.5 cm, laterally 100 cm)
        n = n_hist or 10_000_000
        rho = [1.0] * 3 + [0.0012] * 20 + [1.0] * 4
        return dict(name=name, phantom=slab_phantom(len(rho), 0.5, rho),
                    sources=[pencil(1, 2.0, (50.0, 50.0, 0.0), n)],
                    transport=transport(10.0, 200), seed=1, material=WATER)
    raise KeyError(name)
