"""Workload parameters of the synthetic stand-ins for the paper's examples.

Lengths are in wavelengths (lambda = 1, wavenumber k = 2 pi).  The angular grids
are written out as integers; ``tests/test_oracle_geometry.py`` checks them against the
sampling rule of Section II.A as the oracle implements it (n_theta = L + 1,
n_phi = 2 L + 1, L from the box's enclosing radius and the FMM accuracy).

A sphere workload is a geodesic sphere of diameter ``diameter`` meshed with
frequency ``freq`` (``30 freq^2`` basis functions), grouped by a cubic box grid of
edge ``box`` anchored at the sphere's bounding-box corner (-R, -R, -R) with
``ceil(diameter / box)`` boxes per axis.  A trihedral workload is the corner
reflector of three square plates of side ``diameter`` meshed with ``freq`` squares
per side (``9 freq^2 - 3 freq`` basis functions), its box grid anchored at the
corner (0, 0, 0).
"""
import math
from dataclasses import dataclass, field


@dataclass(frozen=True)
class Workload:
    name: str
    diameter: float
    freq: int
    box: float
    n_theta: int
    n_phi: int
    gamma: float
    nrhs: int = 1
    seeds: dict = field(default_factory=dict)
    shape: str = "sphere"

    @property
    def radius(self):
        return 0.5 * self.diameter

    @property
    def k(self):
        return 2.0 * math.pi

    @property
    def n_basis(self):
        if self.shape == "trihedral":
            return 9 * self.freq * self.freq - 3 * self.freq
        return 30 * self.freq * self.freq

    @property
    def boxes_per_axis(self):
        return int(math.ceil(self.diameter / self.box - 1e-12))

    @property
    def origin(self):
        if self.shape == "trihedral":
            return (0.0, 0.0, 0.0)
        r = self.radius
        return (-r, -r, -r)

    def mesh(self):
        """``(vertices, triangles)`` of the workload's surface."""
        from .mesh import icosphere, trihedral
        if self.shape == "trihedral":
            return trihedral(self.diameter, self.freq)
        return icosphere(self.freq, self.radius)


# Small workload: 1-wavelength sphere, 1280 triangles, 1920 basis functions,
# box 0.5 lambda; grid from L = kd + 1.8 (3)^(2/3) (kd)^(1/3) with d the box
# diagonal, rounded up (L = 13), n_theta = L + 1, n_phi = 2 (L + 1).
SMALL = Workload("sphere-1lambda-f8-box0.5", 1.0, 8, 0.5, 14, 28, 1e-6,
                 seeds={"x": 0, "g": 1})

# The paper's 30-lambda sphere at box 2 lambda, 5 digits: L = 37, a 38 x 75 grid
# (Table IV), 939,870 basis functions in 1034 groups.
SPHERE30 = Workload("sphere-30lambda-f177-box2-grid38x75", 30.0, 177, 2.0, 38, 75, 1e-6,
                    seeds={"x": 0, "g": 1})
# The same sphere on the coarser 29 x 58 grid.
SPHERE30_G29 = Workload("sphere-30lambda-f177-box2-grid29x58", 30.0, 177, 2.0, 29, 58, 1e-6,
                        seeds={"x": 0, "g": 1})

# Mid-size sphere used for fast parity runs at the paper's grid (box 2 lambda).
SPHERE6 = Workload("sphere-6lambda-f36-box2-grid38x75", 6.0, 36, 2.0, 38, 75, 1e-6,
                   seeds={"x": 0, "g": 1})

# Batching workload: 20-lambda sphere, 64 right-hand sides, one box size per run.
SPHERE20 = {
    0.5: Workload("sphere-20lambda-f120-box0.5-grid17x33", 20.0, 120, 0.5, 17, 33, 1e-6, 64, {"x": 2, "g": 1}),
    1.0: Workload("sphere-20lambda-f120-box1-grid25x49", 20.0, 120, 1.0, 25, 49, 1e-6, 64, {"x": 2, "g": 1}),
    2.0: Workload("sphere-20lambda-f120-box2-grid38x75", 20.0, 120, 2.0, 38, 75, 1e-6, 64, {"x": 2, "g": 1}),
    4.0: Workload("sphere-20lambda-f120-box4-grid64x127", 20.0, 120, 4.0, 64, 127, 1e-6, 64, {"x": 2, "g": 1}),
}

# Large Tucker-only workload: 45-lambda sphere, 2,301,870 basis functions.
SPHERE45 = Workload("sphere-45lambda-f277-box2-grid38x75", 45.0, 277, 2.0, 38, 75, 1e-5, 32,
                    {"x": 3, "sample": 4})

# The paper's second example: a trihedral corner reflector of three 6-lambda plates
# (Section III.A; the paper meshes it with 42,477 basis functions, here 69 squares
# per side give 42,642), box 2 lambda (19 non-empty boxes of the 3 x 3 x 3 grid),
# 38 x 75 grid (L = 37, the grid of its Table I memory figure).
TRIHEDRAL = Workload("trihedral-6lambda-n69-box2-grid38x75", 6.0, 69, 2.0, 38, 75, 1e-6,
                     seeds={"x": 0, "g": 1}, shape="trihedral")
# Small trihedral for CPU checks: 2-lambda plates, 12 squares per side (1260 basis
# functions), box 1 lambda (7 groups), 25 x 49 grid (L = 24).
TRIHEDRAL_SMALL = Workload("trihedral-2lambda-n12-box1-grid25x49", 2.0, 12, 1.0, 25, 49, 1e-6,
                           seeds={"x": 0, "g": 1}, shape="trihedral")

ALL = {w.name: w for w in [SMALL, SPHERE30, SPHERE30_G29, SPHERE6, SPHERE45, *SPHERE20.values(),
                           TRIHEDRAL, TRIHEDRAL_SMALL]}
