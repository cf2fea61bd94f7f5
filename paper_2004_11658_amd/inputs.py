"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds no arithmetic of the Deep Potential method itself: it only draws
random numbers (numpy PCG64) and lays them out as
  * model files (architecture + seeded random weights, binary format below),
  * atomic configurations (water lattices, copper FCC, ragged water batches),
  * Maxwell-Boltzmann velocities.

Stand-ins for the paper's systems (Section 4): the trained water / copper models and the
equilibrated 192-atom water cell are not available, so seeded random weights and lattice
water of the same shapes (rc 6 A, N_m 138, nets 25x50x100 / 240^3; copper FCC
a = 3.634 A, rc 8 A) replace them.

Model file format ("DPSEMDL1", little endian)
---------------------------------------------
    off  0  char[8]  magic  b"DPSEMDL1"
    off  8  int32    version (= 1)
    off 12  int32    header_bytes (offset of the first parameter, multiple of 8)
    off 16  int64    nparams
    off 24  int32    ntypes
    off 28  int32    n_emb        embedding layers incl. the first (scalar -> w0) layer
    off 32  int32    n_fit        hidden fitting layers
    off 36  int32    m2           M^< (columns of G kept for the second descriptor factor)
    off 40  int32    switch_kind  0 = C2 quintic, 1 = cosine
    off 44  int32    desc_norm    0 = divide G^T R by N_m, 1 = no normalisation
    off 48  float64  rc
    off 56  float64  rcs          (rc_smth)
    off 64  int32    emb_width[n_emb], fit_width[n_fit], sel[ntypes]
    header_bytes: float64 params[nparams]

Parameter order (this flat order is also the parameter vector theta):
    for a in types, for b in types: embedding net (a, b)
        layer 0: W[1][w0], b[w0]; layer k: W[w_{k-1}][w_k] row major, b[w_k]
    for a in types: fitting net a
        layer 1: W[M*m2][f0], b[f0]; layer k: W[f_{k-1}][f_k], b[f_k]
        output : w[f_last], b[1]
"""
from __future__ import annotations

import dataclasses
import math
import struct
from typing import List, Sequence, Tuple

import numpy as np

MAGIC = b"DPSEMDL1"

# metal units: 1 amu*A^2/fs^2 in eV, and Boltzmann's constant in eV/K
AMU_A2_FS2_IN_EV = 1.0 / 9.64853321e-3
KB_EV = 8.617333262e-5
MASS = {"O": 15.9994, "H": 1.00794, "Cu": 63.546}


@dataclasses.dataclass(frozen=True)
class ModelSpec:
    ntypes: int
    emb_width: Tuple[int, ...]
    fit_width: Tuple[int, ...]
    m2: int
    sel: Tuple[int, ...]
    rc: float
    rcs: float
    switch_kind: int = 0
    desc_norm: int = 0

    @property
    def M(self) -> int:
        return self.emb_width[-1]

    @property
    def nm(self) -> int:
        return int(sum(self.sel))

    def layer_shapes(self):
        """(kind, a, b, n_in, n_out) for every weight block, in file order."""
        out = []
        for a in range(self.ntypes):
            for b in range(self.ntypes):
                n_in = 1
                for w in self.emb_width:
                    out.append(("emb", a, b, n_in, w))
                    n_in = w
        for a in range(self.ntypes):
            n_in = self.M * self.m2
            for w in self.fit_width:
                out.append(("fit", a, -1, n_in, w))
                n_in = w
            out.append(("out", a, -1, n_in, 1))
        return out

    @property
    def nparams(self) -> int:
        return int(sum(i * o + o for (_, _, _, i, o) in self.layer_shapes()))


WATER = ModelSpec(ntypes=2, emb_width=(25, 50, 100), fit_width=(240, 240, 240), m2=16,
                  sel=(46, 92), rc=6.0, rcs=0.5)
COPPER = ModelSpec(ntypes=1, emb_width=(32, 64, 128), fit_width=(240, 240, 240), m2=16,
                   sel=(512,), rc=8.0, rcs=2.0)


def random_params(spec: ModelSpec, seed: int) -> np.ndarray:
    """Seeded random weights.

    Biases ~ N(0, 1) (output bias 0).  Weights ~ N(0, 1/(n_in + n_out)), except the
    embedding nets' first layer, W ~ N(0, 1), so G varies over the range of s, and the
    fitting nets' first layer, W ~ N(0, 2^2): the normalised descriptor entries are
    ~1e-2 (the formulas carry no input standardisation), and narrower weights would
    leave E almost independent of the geometry.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    chunks = []
    for kind, _a, _b, n_in, n_out in spec.layer_shapes():
        std = math.sqrt(1.0 / (n_in + n_out))
        if kind == "emb" and n_in == 1:
            std = 1.0
        elif kind == "fit" and n_in == spec.M * spec.m2:
            std = 2.0
        w = rng.normal(0.0, std, size=(n_in, n_out))
        if kind == "out":
            b = np.zeros(n_out)
        else:
            b = rng.normal(0.0, 1.0, size=n_out)
        chunks += [w.ravel(), b]
    p = np.concatenate(chunks).astype(np.float64)
    assert p.size == spec.nparams
    return p


def model_bytes(spec: ModelSpec, params: np.ndarray) -> bytes:
    ints = list(spec.emb_width) + list(spec.fit_width) + list(spec.sel)
    hdr = MAGIC + struct.pack("<iiq", 1, 0, spec.nparams)
    hdr += struct.pack("<iiiiii", spec.ntypes, len(spec.emb_width), len(spec.fit_width),
                       spec.m2, spec.switch_kind, spec.desc_norm)
    hdr += struct.pack("<dd", spec.rc, spec.rcs)
    hdr += struct.pack("<%di" % len(ints), *ints)
    hb = (len(hdr) + 7) // 8 * 8
    hdr = hdr + b"\0" * (hb - len(hdr))
    hdr = hdr[:12] + struct.pack("<i", hb) + hdr[16:]
    assert params.dtype == np.float64 and params.size == spec.nparams
    return hdr + params.astype("<f8").tobytes()


def write_model(path: str, spec: ModelSpec, params: np.ndarray) -> str:
    with open(path, "wb") as f:
        f.write(model_bytes(spec, params))
    return path


# ---------------------------------------------------------------------------------------
# configurations
# ---------------------------------------------------------------------------------------

def _rand_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def _min_image_dist(a: np.ndarray, b: np.ndarray, L: float) -> np.ndarray:
    d = b[None, :, :] - a[:, None, :]
    d -= L * np.round(d / L)
    return np.sqrt((d * d).sum(-1))


def water_lattice(n_side: Sequence[int] | int, L: float, seed: int, n_mol: int | None = None,
                  jitter: float = 0.3, roh: float = 0.96, hoh_deg: float = 104.5,
                  min_dist: float = 1.0):
    """Water molecules on a cubic lattice in a periodic cube of side L.

    O at lattice sites + U(-jitter, jitter) per component, random SO(3) orientation,
    rigid O-H = roh and H-O-H = hoh_deg; an orientation is redrawn while any
    intermolecular distance falls below min_dist.  If n_mol is given, n_mol of the
    n_side^3 sites are drawn at random.  Atom order: all O, then all H (molecule-major).
    Returns coords [N][3] float64, types [N] int32 (O = 0, H = 1), box [3][3].
    """
    if isinstance(n_side, int):
        n_side = (n_side, n_side, n_side)
    rng = np.random.Generator(np.random.PCG64(seed))
    sites = np.array([(i, j, k) for i in range(n_side[0]) for j in range(n_side[1])
                      for k in range(n_side[2])], dtype=np.float64)
    if n_mol is not None and n_mol < len(sites):
        sel = np.sort(rng.choice(len(sites), size=n_mol, replace=False))
        sites = sites[sel]
    nm = len(sites)
    a = np.array([L / n_side[0], L / n_side[1], L / n_side[2]])
    O = (sites + 0.5) * a + rng.uniform(-jitter, jitter, size=(nm, 3))
    half = math.radians(hoh_deg) / 2.0
    body = np.array([[roh * math.cos(half), roh * math.sin(half), 0.0],
                     [roh * math.cos(half), -roh * math.sin(half), 0.0]])
    H = np.zeros((nm, 2, 3))
    # only molecules on neighbouring lattice sites (+-1 per axis) can come within
    # min_dist: two sites apart the O-O distance exceeds 2 spacings - 2 jitters
    grid = -np.ones(tuple(n_side), dtype=np.int64)
    isites = sites.astype(np.int64)
    grid[isites[:, 0], isites[:, 1], isites[:, 2]] = np.arange(nm)
    done = np.zeros(nm, dtype=bool)
    offs = np.array([(i, j, k) for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)
                     if (i, j, k) != (0, 0, 0)])
    for m in range(nm):
        nb = (isites[m][None, :] + offs) % np.asarray(n_side)
        ids = np.unique(grid[nb[:, 0], nb[:, 1], nb[:, 2]])
        ids = ids[(ids >= 0) & (ids != m)]
        others = [O[ids]]
        dn = ids[done[ids]]
        if dn.size:
            others.append(H[dn].reshape(-1, 3))
        others = np.vstack(others)
        for _try in range(200):
            Q = _rand_rotation(rng)
            h = O[m] + body @ Q.T
            if others.shape[0] == 0:
                break
            mol = np.vstack([O[m][None], h])
            if _min_image_dist(mol, others, L).min() >= min_dist:
                break
        H[m] = h
        done[m] = True
    coords = np.vstack([O, H.reshape(-1, 3)])
    types = np.concatenate([np.zeros(nm, np.int32), np.ones(2 * nm, np.int32)])
    box = np.diag([L, L, L]).astype(np.float64)
    return coords.astype(np.float64), types, box


def copper_fcc(n_cells: int, a: float, seed: int, sigma: float = 0.1):
    """FCC copper, n_cells^3 conventional cells of side a, N(0, sigma) jitter per component."""
    rng = np.random.Generator(np.random.PCG64(seed))
    basis = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    g = np.arange(n_cells)
    cells = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pos = ((cells[:, None, :] + basis[None]) * a).reshape(-1, 3)
    pos = pos + rng.normal(0.0, sigma, size=pos.shape)
    L = n_cells * a
    return pos.astype(np.float64), np.zeros(len(pos), np.int32), np.diag([L, L, L]).astype(np.float64)


def maxwell_velocities(types: np.ndarray, masses: Sequence[float], T: float, seed: int):
    """v ~ N(0, kB T / m) per component (A/fs), centre-of-mass momentum removed, then
    rescaled so the kinetic temperature over 3N-3 degrees of freedom is exactly T."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = np.asarray(masses, np.float64)[types]
    sig = np.sqrt(KB_EV * T / (m * AMU_A2_FS2_IN_EV))
    v = rng.normal(size=(len(types), 3)) * sig[:, None]
    p = (m[:, None] * v).sum(0)
    v -= p / m.sum()
    ke = 0.5 * AMU_A2_FS2_IN_EV * (m[:, None] * v * v).sum()
    t_now = 2.0 * ke / ((3 * len(types) - 3) * KB_EV)
    v *= math.sqrt(T / t_now)
    return v


# ---------------------------------------------------------------------------------------
# the benchmark / test workloads
# ---------------------------------------------------------------------------------------

WATER_DENSITY_MOL_PER_A3 = 0.033405


def config_water192(seed: int = 201):
    """64 H2O on a 4^3 lattice in a 12.42 A cube (192 atoms)."""
    return water_lattice(4, 12.42, seed)


def config_water12k(seed: int = 202):
    """4096 H2O on a 16^3 lattice in a 49.7 A cube (12,288 atoms)."""
    return water_lattice(16, 49.7, seed)


def config_copper131k(seed: int = 203):
    """Cu FCC 32^3 cells, a = 3.634 A (131,072 atoms)."""
    return copper_fcc(32, 3.634, seed)


def config_water786k(seed: int = 205):
    """262,144 H2O on a 64^3 lattice in a 197.9 A cube (786,432 atoms)."""
    return water_lattice(64, 197.9, seed)


def ragged_water_batch(nframes: int = 64, seed: int = 204, nmol_lo: int = 32,
                       nmol_hi: int = 1024) -> List[tuple]:
    """nframes water frames, n_mol ~ U{nmol_lo..nmol_hi}, box side from liquid density,
    n_mol of ceil(n_mol^(1/3))^3 lattice sites drawn at random."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nmols = rng.integers(nmol_lo, nmol_hi + 1, size=nframes)
    frames = []
    for f, n in enumerate(nmols):
        L = (n / WATER_DENSITY_MOL_PER_A3) ** (1.0 / 3.0)
        side = int(math.ceil(n ** (1.0 / 3.0) - 1e-9))
        frames.append(water_lattice(side, L, seed * 1000 + f, n_mol=int(n)))
    return frames


def small_water(n_side: int, L: float, seed: int):
    """A small water box (used for multi-image / small-box cases)."""
    return water_lattice(n_side, L, seed)
