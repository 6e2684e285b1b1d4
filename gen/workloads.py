"""Seeded synthetic workloads shaped like the paper's bcc-W simulations.

This module draws inputs only: atom positions, species, velocities, region
shapes and the random coefficients of the two synthetic potentials. It holds
none of the method's arithmetic (no neighbour search, region weight, basis
function, energy or force). Both the FP64 oracle and the HIP library read the
same dictionaries it returns.

Units: Angstrom, eV, amu, fs.

Workload recipes (the paper's trained potentials and datasets are not used;
these stand in for the shapes of its case studies):
  c1  5x5x5 bcc W cells, one vacancy at the box centre, sigma 0.05 A,
      FP64; sphere 6 A core + 2 A linear blend, 5 A buffer.
  c2  16x16x16 bcc W cells with a <111> dumbbell replacing the corner atom at
      (8a,8a,8a), sigma 0.08 A; sphere 8 + 2 A at the dumbbell centre.
  c3  54,000-atom [1-01]x[-12-1]x[111] column, periodic along z only, with a
      1/2[111] screw dislocation (u_z = b*theta/2pi); z-cylinder 12 + 3 A.
  c4  W(001) slab replicas (14x14 cells laterally) with one He atom 6 A above
      the surface at 10-80 eV, +-5 degrees from the normal; sphere 6 + 2 A
      following the He atom.
  c5  80x80x80 bcc W cells with 200 random vacancies, sigma 0.05 A; a 7 + 2 A
      sphere at each vacancy.
"""
import numpy as np

from .lattice import A_W, bcc_cubic, screw_cell, replicate, wrap

KAPPA = 9.648533212e-3      # (eV/A)/amu expressed in A/fs^2
KB = 8.617333262e-5         # eV/K
MASS = {0: 183.84, 1: 4.002602}   # species 0 = W, species 1 = He
BASE_SEED = 2502190810

# Scales of the random linear coefficients, one per correlation order, and of
# the cheap spline coefficients. They were fixed once so that, on each
# workload's displaced lattice, every correlation order contributes a force of
# order 1 eV/A (the random draws are otherwise unscaled N(0,1)).
ACE_SCALE = {
    "c1": (0.6, 0.3, 0.0),
    "c2": (0.2, 0.02, 0.01),
    # MD workloads: 20x weaker random parts (forces ~0.05 eV/A) so that the
    # 1-ps runs stay near the crystal instead of collapsing
    "c3": (0.01, 0.001, 0.0005),
    "c4": (0.025, 0.0075, 0.003),
    "c5": (0.3, 0.008, 0.017),
    "tiny": (1.7, 2.8, 1.9),
}
UF3_SCALE2 = 0.1   # "coefficients N(0, 0.1)": standard deviation 0.1 eV
UF3_SCALE3 = 0.02


def _streams(seed, n=8):
    ss = np.random.SeedSequence(seed)
    return [np.random.default_rng(s) for s in ss.spawn(n)]


def ace_params(rng, n_species, n_rad, lmax, order, rcut, scales):
    """Dense random coefficient arrays of the ACE-style model.

    c1[z][a], c2[z][l][a][b] (entries a<=b are read), c3[z][p][q][r] with
    p = a*(lmax+1)+l (entries p<=q<=r are read); a = species*n_rad + n.
    """
    nchan = n_species * n_rad
    K = nchan * (lmax + 1)
    s1, s2, s3 = scales
    c0 = rng.normal(0.0, 1.0, size=(n_species,))
    c1 = rng.normal(0.0, 1.0, size=(n_species, nchan)) * s1
    c2 = rng.normal(0.0, 1.0, size=(n_species, lmax + 1, nchan, nchan)) * s2
    if order >= 3:
        c3 = rng.normal(0.0, 1.0, size=(n_species, K, K, K)) * s3
    else:
        c3 = np.zeros((n_species, 1, 1, 1))
    return dict(n_rad=n_rad, lmax=lmax, order=order, rcut=float(rcut),
                c0=c0, c1=c1, c2=c2, c3=c3)


def uf3_params(rng, n_species, n_knots2, rcut2, n_knots3=0, rcut3=3.5,
               scale2=UF3_SCALE2, scale3=UF3_SCALE3):
    """Random clamped-cubic-B-spline coefficients.

    c2[zi][zj][n] (symmetric in zi, zj), n_knots2 + 2 coefficients per pair,
    the last three zero so that V2 vanishes smoothly at rcut2.
    c3[z][p][q][s] with n_knots3 + 2 per axis, symmetric in (p, q), the last
    three along p and along q zero so that V3 vanishes smoothly at rcut3.
    """
    nb2 = n_knots2 + 2
    c2 = np.zeros((n_species, n_species, nb2))
    for a in range(n_species):
        for b in range(a, n_species):
            v = rng.normal(0.0, scale2, size=nb2)
            v[-3:] = 0.0
            c2[a, b] = v
            c2[b, a] = v
    if n_knots3 > 0:
        nb3 = n_knots3 + 2
        c3 = rng.normal(0.0, scale3, size=(n_species, nb3, nb3, nb3))
        c3 = 0.5 * (c3 + c3.transpose(0, 2, 1, 3))
        c3[:, -3:, :, :] = 0.0
        c3[:, :, -3:, :] = 0.0
    else:
        c3 = np.zeros((n_species, 1, 1, 1))
    return dict(n_knots2=n_knots2, rcut2=float(rcut2), c2=c2,
                n_knots3=n_knots3, rcut3=float(rcut3), c3=c3)


def sphere(center, r_core, r_blend, follow_atom=-1, blend=0):
    return dict(type=0, axis=2, follow_atom=int(follow_atom),
                center=np.asarray(center, dtype=np.float64), r_core=float(r_core),
                r_blend=float(r_blend), blend=int(blend))


def cylinder(center, axis, r_core, r_blend, blend=0):
    return dict(type=1, axis=int(axis), follow_atom=-1,
                center=np.asarray(center, dtype=np.float64), r_core=float(r_core),
                r_blend=float(r_blend), blend=int(blend))


def seeded(r_core, r_blend, blend=0):
    """Seeded region (the paper's fix): core = seed atoms and their neighbours
    within r_core, blend measured to the nearest core atom; the seeds are the
    workload's boolean array w["seeds"]."""
    return dict(type=2, axis=2, follow_atom=-1, center=np.zeros(3), r_core=float(r_core),
                r_blend=float(r_blend), blend=int(blend))


def maxwell(rng, species, T):
    m = np.array([MASS[int(s)] for s in species])
    sig = np.sqrt(KAPPA * KB * T / m)
    v = rng.normal(0.0, 1.0, size=(len(species), 3)) * sig[:, None]
    vcm = (m[:, None] * v).sum(0) / m.sum()
    return v - vcm[None, :]


def _pack(name, seed, pos, species, L, periodic, regions, r_buffer, model, **extra):
    d = dict(name=name, seed=seed, pos=np.ascontiguousarray(pos, dtype=np.float64),
             species=np.ascontiguousarray(species, dtype=np.int32),
             L=np.asarray(L, dtype=np.float64), periodic=np.asarray(periodic, dtype=np.int32),
             regions=regions, r_buffer=float(r_buffer), model=model,
             masses=np.array([MASS[0], MASS[1]]))
    d.update(extra)
    return d


def c1(seed=BASE_SEED + 0, sigma=0.05):
    r = _streams(seed)
    n = 5
    pos = bcc_cubic(n, n, n)
    L = np.array([n * A_W] * 3)
    centre = np.array([2.5 * A_W] * 3)
    keep = np.linalg.norm(pos - centre, axis=1) > 1e-6
    pos = pos[keep]
    pos = pos + r[0].normal(0.0, sigma, size=pos.shape)
    pos = wrap(pos, L, [1, 1, 1])
    species = np.zeros(len(pos), dtype=np.int32)
    model = dict(n_species=1, skin=1.0,
                 ace=ace_params(r[1], 1, 8, 3, 2, 5.0, ACE_SCALE["c1"]),
                 uf3=uf3_params(r[2], 1, 12, 5.0))
    return _pack("c1", seed, pos, species, L, [1, 1, 1],
                 [sphere(centre, 6.0, 2.0)], 5.0, model, precision="fp64")


def c2_model(rng_ace, rng_uf3, n_species=1, rcut_exp=5.5, scales=None, uf3_scale=1.0):
    return dict(n_species=n_species, skin=1.0,
                ace=ace_params(rng_ace, n_species, 12, 4, 3, rcut_exp,
                               scales or ACE_SCALE["c2"]),
                uf3=uf3_params(rng_uf3, n_species, 16, 5.5, 6, 3.5,
                               UF3_SCALE2 * uf3_scale, UF3_SCALE3 * uf3_scale))


def c2(seed=BASE_SEED + 1, sigma=0.08):
    r = _streams(seed)
    n = 16
    pos = bcc_cubic(n, n, n)
    L = np.array([n * A_W] * 3)
    corner = np.array([8 * A_W] * 3)
    k = int(np.argmin(np.linalg.norm(pos - corner, axis=1)))
    d = (A_W / 8.0) * np.ones(3)
    pos = np.concatenate([np.delete(pos, k, axis=0), (corner + d)[None], (corner - d)[None]])
    pos = pos + r[0].normal(0.0, sigma, size=pos.shape)
    pos = wrap(pos, L, [1, 1, 1])
    species = np.zeros(len(pos), dtype=np.int32)
    model = c2_model(r[1], r[2])
    return _pack("c2", seed, pos, species, L, [1, 1, 1],
                 [sphere(corner, 8.0, 2.0)], 5.5, model, precision="fp32")


def c3(seed=BASE_SEED + 2, T=300.0, margin=12.0, ncell=(30, 15, 20)):
    r = _streams(seed)
    cell, edges = screw_cell()
    pos = replicate(cell, edges, *ncell)
    ext = edges * np.array(ncell)
    b = np.sqrt(3.0) * A_W / 2.0
    core = np.array([ext[0] / 2 + 0.1, ext[1] / 2 + 0.1])
    theta = np.arctan2(pos[:, 1] - core[1], pos[:, 0] - core[0])
    pos[:, 2] += b * theta / (2.0 * np.pi)
    L = np.array([ext[0] + 2 * margin, ext[1] + 2 * margin, ext[2]])
    pos[:, 0] += margin
    pos[:, 1] += margin
    pos = wrap(pos, L, [0, 0, 1])
    species = np.zeros(len(pos), dtype=np.int32)
    model = c2_model(r[1], r[2], scales=ACE_SCALE["c3"], uf3_scale=0.05)
    vel = maxwell(r[3], species, T)
    centre = np.array([core[0] + margin, core[1] + margin, 0.0])
    return _pack("c3", seed, pos, species, L, [0, 0, 1],
                 [cylinder(centre, 2, 12.0, 3.0)], 5.5, model, vel=vel,
                 precision="fp32", dt=1.0, T=T)


HE_WALL = 100.0  # eV; weight of the smooth He-W repulsion in both potentials


def c4_model(seed=BASE_SEED + 3):
    """Two species (W = 0, He = 1). Random weak parts as the other MD
    workload, plus a smooth He-W repulsion in both potentials so that 10-80 eV
    He atoms reflect or stop: in the ACE-style model the order-1 weight of the
    n = 0 radial function of the unlike channel (R_0 is the decreasing
    envelope), in the UF3-style model a decreasing ramp on the He-W pair
    spline."""
    r = _streams(seed)
    ace = ace_params(r[1], 2, 12, 4, 3, 5.0, ACE_SCALE["c4"])
    nr = ace["n_rad"]
    ace["c1"][0, 1 * nr + 0] = HE_WALL   # W centre, He neighbours
    ace["c1"][1, 0 * nr + 0] = HE_WALL   # He centre, W neighbours
    uf3 = uf3_params(r[2], 2, 16, 6.0, 6, 3.5, UF3_SCALE2 * 0.05, UF3_SCALE3 * 0.05)
    nb2 = uf3["c2"].shape[-1]
    ramp = np.maximum(0.0, 1.0 - np.arange(nb2) / 7.0) ** 2 * 20.0
    ramp[-3:] = 0.0
    uf3["c2"][0, 1] += ramp
    uf3["c2"][1, 0] += ramp
    return dict(n_species=2, skin=1.0, ace=ace, uf3=uf3)


def c4_replica(index, seed=BASE_SEED + 3, n_min=2000, n_max=20000, T=1000.0,
               vacuum_above=300.0, vacuum_below=20.0, n_target=None):
    """One W(001)+He impact replica. Replicas share the model of c4_model."""
    rs = np.random.default_rng(np.random.SeedSequence([seed, 7919, index]))
    if n_target is None:
        n_target = float(np.exp(rs.uniform(np.log(n_min), np.log(n_max))))
    m = max(2, int(round(n_target / 392.0)))
    pos = bcc_cubic(14, 14, m)
    Lx = 14 * A_W
    top = pos[:, 2].max()
    pos[:, 2] += vacuum_below
    top += vacuum_below
    he = np.array([rs.uniform(0, Lx), rs.uniform(0, Lx), top + 6.0])
    pos = np.concatenate([pos, he[None]])
    species = np.zeros(len(pos), dtype=np.int32)
    species[-1] = 1
    L = np.array([Lx, Lx, top + vacuum_above])
    pos = wrap(pos, L, [1, 1, 0])
    vel = maxwell(rs, species, T)
    E = rs.uniform(10.0, 80.0)
    pol = np.deg2rad(rs.uniform(0.0, 5.0))
    az = rs.uniform(0.0, 2 * np.pi)
    speed = np.sqrt(2.0 * E * KAPPA / MASS[1])
    vel[-1] = speed * np.array([np.sin(pol) * np.cos(az), np.sin(pol) * np.sin(az), -np.cos(pol)])
    he_idx = len(pos) - 1
    return _pack("c4", seed, pos, species, L, [1, 1, 0],
                 [sphere(he, 6.0, 2.0, follow_atom=he_idx)], 5.0, c4_model(seed),
                 vel=vel, precision="fp32", dt=0.2, T=T, he_energy=E, replica=index)


def c5(seed=BASE_SEED + 4, sigma=0.05, n=80, n_vac=200):
    r = _streams(seed)
    pos = bcc_cubic(n, n, n)
    L = np.array([n * A_W] * 3)
    vac = r[4].choice(len(pos), size=n_vac, replace=False)
    centres = pos[np.sort(vac)]
    pos = np.delete(pos, vac, axis=0)
    pos = pos + r[0].normal(0.0, sigma, size=pos.shape)
    pos = wrap(pos, L, [1, 1, 1])
    species = np.zeros(len(pos), dtype=np.int32)
    model = dict(n_species=1, skin=1.0,
                 ace=ace_params(r[1], 1, 16, 5, 3, 5.0, ACE_SCALE["c5"]),
                 uf3=uf3_params(r[2], 1, 16, 5.5, 6, 3.5))
    regions = [sphere(c, 7.0, 2.0) for c in centres]
    return _pack("c5", seed, pos, species, L, [1, 1, 1], regions, 5.0, model,
                 precision="fp32", vacancy_centres=centres)


def subvolume(w, centre, edge):
    """Indices of atoms inside a cube (minimum image) of the given edge."""
    d = w["pos"] - np.asarray(centre)[None, :]
    for k in range(3):
        if w["periodic"][k]:
            d[:, k] -= w["L"][k] * np.round(d[:, k] / w["L"][k])
    return np.nonzero(np.all(np.abs(d) < edge / 2.0, axis=1))[0].astype(np.int64)


def tiny(seed=12345, n_species=1, order=3, lmax=3, n_rad=4, cells=3, sigma=0.1,
         periodic=(1, 1, 1), rcut=4.2, three_body=True, vacuum=0.0):
    """Small cell for oracle pins and quick parity runs."""
    r = _streams(seed)
    pos = bcc_cubic(cells, cells, cells)
    L = np.array([cells * A_W] * 3)
    for k in range(3):
        if not periodic[k]:
            pos[:, k] += vacuum
            L[k] += 2 * vacuum
    pos = pos + r[0].normal(0.0, sigma, size=pos.shape)
    pos = wrap(pos, L, periodic)
    species = r[5].integers(0, n_species, size=len(pos)).astype(np.int32)
    model = dict(n_species=n_species, skin=0.5,
                 ace=ace_params(r[1], n_species, n_rad, lmax, order, rcut, ACE_SCALE["tiny"]),
                 uf3=uf3_params(r[2], n_species, 8, rcut, 4 if three_body else 0, 3.2))
    centre = L / 2.0
    return _pack("tiny", seed, pos, species, L, periodic,
                 [sphere(centre, 2.5, 1.5)], 2.5, model, precision="fp64",
                 vel=maxwell(r[3], species, 300.0))
