"""Synthetic data for the constrained linear fit of the cheap potential.

Geometry only: thermal snapshots of bulk bcc W (soft constraints) and
homogeneously strained bulk cells (hard constraints), following the recipe of
the paper's "Generation of synthetic data" (Methods): soft data = energies and
forces of high-temperature bulk snapshots, hard data = energies of 17 strains
in +-0.5 % for each of six strain states. Labels are computed elsewhere with
the expensive potential; nothing here evaluates a potential.

Strain states. The paper's list (hydrostatic, uniaxial [100], uniaxial [111],
and three simple shears) needs sheared, non-orthorhombic cells for the shears;
the boxes here are orthorhombic, so the shears are replaced by strains that
are diagonal in a rotated orthorhombic cell and still separate the three
cubic elastic constants: pure shear in the (x=[110], y=[-110]) frame (C44),
uniaxial [110] ((C11+C12+2 C44)/2) and the tetragonal shear diag(1+e/2,
1-e/2, 1) ((C11-C12)/2), beside hydrostatic (C11+2 C12), uniaxial [100]
(C11) and uniaxial [111] ((C11+2 C12+4 C44)/3).
"""
import numpy as np

from gen.lattice import A_W, bcc_cubic, oriented_bcc, replicate, wrap

CUBIC = ((1, 0, 0), (0, 1, 0), (0, 0, 1))
FRAME110 = ((1, 1, 0), (-1, 1, 0), (0, 0, 1))
FRAME111 = ((1, 0, -1), (-1, 2, -1), (1, 1, 1))


def _cell(frame):
    if frame == "cubic":
        return bcc_cubic(5, 5, 5), np.full(3, 5 * A_W)
    if frame == "110":
        c, e = oriented_bcc(*FRAME110, periods=(np.sqrt(2.0), np.sqrt(2.0), 1.0))
        return replicate(c, e, 3, 3, 5), e * np.array([3, 3, 5])
    c, e = oriented_bcc(*FRAME111, periods=(np.sqrt(2.0), np.sqrt(6.0), np.sqrt(3.0) / 2.0))
    return replicate(c, e, 3, 2, 6), e * np.array([3, 2, 6])


# (name, cell frame, diagonal stretch factors as functions of the strain e)
STRAIN_STATES = (
    ("hydrostatic", "cubic", lambda e: (1 + e, 1 + e, 1 + e)),
    ("uniaxial [100]", "cubic", lambda e: (1 + e, 1.0, 1.0)),
    ("uniaxial [111]", "111", lambda e: (1.0, 1.0, 1 + e)),
    ("pure shear [110]/[-110] (C44)", "110", lambda e: (1 + e / 2, 1 - e / 2, 1.0)),
    ("uniaxial [110]", "110", lambda e: (1 + e, 1.0, 1.0)),
    ("tetragonal shear", "cubic", lambda e: (1 + e / 2, 1 - e / 2, 1.0)),
)


def strained_cells(n_strain=17, max_strain=0.005):
    """Hard-constraint configurations: list of dict(pos, L, periodic, state, strain)."""
    out = []
    for name, frame, stretch in STRAIN_STATES:
        pos0, L0 = _cell(frame)
        for e in np.linspace(-max_strain, max_strain, n_strain):
            f = np.asarray(stretch(e))
            L = L0 * f
            out.append(dict(pos=wrap(pos0 * f, L, [1, 1, 1]), L=L, periodic=np.ones(3, np.int32),
                            state=name, strain=float(e)))
    return out


def thermal_snapshots(n_snap, cells=10, sigma=0.1, seed=2502190815):
    """Soft-constraint configurations: bulk bcc cubes (2 cells^3 atoms) with
    independent Gaussian displacements of standard deviation sigma (A) per
    coordinate, one seeded stream per snapshot."""
    base = bcc_cubic(cells, cells, cells)
    L = np.full(3, cells * A_W)
    ss = np.random.SeedSequence(seed).spawn(n_snap)
    out = []
    for s in ss:
        r = np.random.default_rng(s)
        out.append(dict(pos=wrap(base + r.normal(0.0, sigma, base.shape), L, [1, 1, 1]), L=L,
                        periodic=np.ones(3, np.int32)))
    return out


def fit_model(seed=2502190816, n_knots2=12, n_knots3=5):
    """Model description for the fit: the expensive potential of the
    8,193-atom W workload (ACE-style, 12 radial functions, lmax 4, order 3,
    5.5 A) labels the data; the cheap potential's shape (clamped cubic
    B-splines, 2-body on [0, 5.5] A with n_knots2 points, 3-body legs on
    [0, 3.5] A with n_knots3 points) fixes the parameters being fitted. Its
    random coefficients are only a starting model."""
    from gen.workloads import ACE_SCALE, _streams, ace_params, uf3_params
    r = _streams(seed)
    return dict(n_species=1, skin=1.0,
                ace=ace_params(r[1], 1, 12, 4, 3, 5.5, ACE_SCALE["c2"]),
                uf3=uf3_params(r[2], 1, n_knots2, 5.5, n_knots3, 3.5))
