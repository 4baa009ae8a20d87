"""Seeded synthetic workloads for the ANI-style energy/force path.

This module only draws inputs: coordinates, species, boxes, network weights
and request traces.  It holds none of the method's arithmetic (no cutoff, no
symmetry function, no network evaluation), so the CPU oracle and the GPU path
can both be fed from it without sharing any of the computation.

Species slots follow the ANI-2x element set (paper, "ANI models"):
0 = H, 1 = C, 2 = N, 3 = O, 4 = S, 5 = F, 6 = Cl.

Every generator returns float32 coordinates: the GPU path computes in float32
and the oracle reads the same float32 values exactly in float64, so the two
sides see bit-identical inputs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

H, C, N, O, S, F, CL = 0, 1, 2, 3, 4, 5, 6
SPECIES_NAMES = ("H", "C", "N", "O", "S", "F", "Cl")
N_SPECIES = 7

# Water: 18.015 g/mol at 1 g/cm^3 -> volume per molecule in A^3.
WATER_VOL_A3 = 18.015 / 0.602214076
OH_BOND = 0.96
HOH_ANGLE_DEG = 104.5


# --------------------------------------------------------------------------
# Model description (hyper-parameters and weights are data, not arithmetic)
# --------------------------------------------------------------------------

def aev_params() -> dict:
    """AEV hyper-parameters of the workloads (7 species -> 1008 features).

    Radial: eta 19.7 A^-2, 16 shifts evenly spaced 0.8..4.9 A inclusive,
    cutoff 5.1 A, prefactor 0.25.  Angular: eta 12.5 A^-2, zeta 14.1,
    4 radial shifts 0.8..2.85 A inclusive, 8 angle shifts pi/16 + k*pi/8,
    cutoff 3.5 A.
    """
    return dict(
        n_species=N_SPECIES,
        rc_rad=5.1, eta_rad=19.7,
        shf_rad=np.linspace(0.8, 4.9, 16),
        rc_ang=3.5, eta_ang=12.5, zeta=14.1,
        shf_ang=np.linspace(0.8, 2.85, 4),
        shf_z=np.pi / 16 + np.arange(8) * np.pi / 8,
        radial_scale=0.25,
    )


# DeepPot-style descriptor (section "DeePMD Models"): neighbours kept per
# species slot, nearest first.  Within 6 A of an atom of water or a solvated
# protein sit about 60 H, 30 O and (protein) 15 C / 4 N.
DP_SEL = (48, 24, 8, 24, 4, 4, 8)


def dp_params(rc: float = 6.0, sel=DP_SEL) -> dict:
    """DeepPot-style descriptor hyper-parameters: cutoff 6 A, at most sel[s]
    neighbours of species s (120 slots, 4 features each -> 480 features)."""
    return dict(kind="dp", n_species=len(sel), rc=float(rc), sel=tuple(int(x) for x in sel))


def aev_dim(p: dict) -> int:
    """Descriptor length of either kind (AEV or DeepPot-style)."""
    if p.get("kind") == "dp":
        return 4 * sum(p["sel"])
    s = p["n_species"]
    return s * len(p["shf_rad"]) + (s * (s + 1) // 2) * len(p["shf_ang"]) * len(p["shf_z"])


# hidden widths per species slot (input width is the AEV length, output 1)
HIDDEN = {
    H: (256, 192, 160),
    C: (224, 192, 160),
    N: (192, 160, 128),
    O: (192, 160, 128),
    S: (160, 128, 96),
    F: (160, 128, 96),
    CL: (160, 128, 96),
}


@dataclass
class ModelSpec:
    """Everything needed to build a network set on either side.

    weights: float32 flat array, concatenated over (member, species, layer),
    each layer stored as W[out][in] followed by b[out].
    """
    aev: dict
    n_ensemble: int
    widths: list  # per species: tuple of layer widths incl. input and output
    weights: np.ndarray
    celu_alpha: float = 0.1

    @property
    def n_species(self) -> int:
        return len(self.widths)

    @property
    def kind(self) -> str:
        """Descriptor kind: "ani" (AEV) or "dp" (DeepPot-style)."""
        return self.aev.get("kind", "ani")

    def layer_slices(self):
        """Yield (member, species, layer, W_slice, b_slice, n_out, n_in)."""
        off = 0
        for m in range(self.n_ensemble):
            for s, w in enumerate(self.widths):
                for l in range(len(w) - 1):
                    n_in, n_out = w[l], w[l + 1]
                    ws = slice(off, off + n_out * n_in)
                    off += n_out * n_in
                    bs = slice(off, off + n_out)
                    off += n_out
                    yield m, s, l, ws, bs, n_out, n_in


def n_params(widths, n_ensemble: int) -> int:
    tot = 0
    for w in widths:
        for l in range(len(w) - 1):
            tot += w[l] * w[l + 1] + w[l + 1]
    return tot * n_ensemble


def make_model(seed: int = 0, n_ensemble: int = 1, hidden=None, aev=None,
               celu_alpha: float = 0.1) -> ModelSpec:
    """Random network set: weights and biases ~ N(0, 1/fan_in), float32.

    Each (member, species, layer) draws from its own stream spawned from
    `seed`, so adding members or species never changes existing weights.
    """
    aev = aev if aev is not None else aev_params()
    d = aev_dim(aev)
    hidden = hidden if hidden is not None else HIDDEN
    widths = [tuple([d] + list(hidden[s]) + [1]) for s in range(aev["n_species"])]
    total = n_params(widths, n_ensemble)
    out = np.empty(total, dtype=np.float32)
    root = np.random.SeedSequence(seed)
    kids = root.spawn(n_ensemble * len(widths))
    off = 0
    k = 0
    for m in range(n_ensemble):
        for s, w in enumerate(widths):
            rng = np.random.Generator(np.random.PCG64(kids[k]))
            k += 1
            for l in range(len(w) - 1):
                n_in, n_out = w[l], w[l + 1]
                std = 1.0 / math.sqrt(n_in)
                cnt = n_out * n_in + n_out
                out[off:off + cnt] = rng.normal(0.0, std, cnt).astype(np.float32)
                off += cnt
    assert off == total
    return ModelSpec(aev=aev, n_ensemble=n_ensemble, widths=widths, weights=out,
                     celu_alpha=celu_alpha)


def make_dp_model(seed: int = 0, n_ensemble: int = 1, hidden=None, dp=None,
                  celu_alpha: float = 0.1) -> ModelSpec:
    """Random network set on the DeepPot-style descriptor (same networks,
    480 inputs)."""
    return make_model(seed, n_ensemble, hidden, dp if dp is not None else dp_params(), celu_alpha)


def linear_readout_model(seed: int = 0, aev=None) -> ModelSpec:
    """Networks with no hidden layer (AEV -> 1): isolates AEV and force work."""
    aev = aev if aev is not None else aev_params()
    return make_model(seed, 1, hidden={s: () for s in range(aev["n_species"])}, aev=aev)


# --------------------------------------------------------------------------
# Systems
# --------------------------------------------------------------------------

@dataclass
class System:
    coords: np.ndarray   # [n, 3] float32
    species: np.ndarray  # [n] int32
    box: np.ndarray      # [3] float32, zeros = non-periodic

    @property
    def n(self) -> int:
        return int(self.coords.shape[0])

    @property
    def periodic(self) -> bool:
        return bool(np.all(self.box > 0))


@dataclass
class Batch:
    coords: np.ndarray    # [N, 3] float32
    species: np.ndarray   # [N] int32
    boxes: np.ndarray     # [S, 3] float32
    offsets: np.ndarray   # [S + 1] int64
    systems: list = field(default_factory=list)

    @property
    def n_atoms(self) -> int:
        return int(self.offsets[-1])

    @property
    def n_systems(self) -> int:
        return int(len(self.offsets) - 1)


def make_batch(systems) -> Batch:
    systems = list(systems)
    offs = np.zeros(len(systems) + 1, dtype=np.int64)
    for k, s in enumerate(systems):
        offs[k + 1] = offs[k] + s.n
    coords = np.concatenate([s.coords for s in systems]).astype(np.float32) if systems else np.zeros((0, 3), np.float32)
    species = np.concatenate([s.species for s in systems]).astype(np.int32) if systems else np.zeros(0, np.int32)
    boxes = np.stack([s.box for s in systems]).astype(np.float32) if systems else np.zeros((0, 3), np.float32)
    return Batch(coords=coords, species=species, boxes=boxes, offsets=offs, systems=systems)


def _rsa(rng, n, lo, hi, dmin, inside=None, max_tries=2000):
    """Random sequential addition in the box [lo, hi)^3 with a minimum distance.

    `inside` optionally restricts candidates (boolean function of a point).
    Returns None if an atom could not be placed within `max_tries` draws.
    """
    pts = np.empty((n, 3), dtype=np.float64)
    cell = dmin
    grid = {}
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    d2 = dmin * dmin
    for k in range(n):
        for _ in range(max_tries):
            p = lo + rng.random(3) * (hi - lo)
            if inside is not None and not inside(p):
                continue
            c = tuple(np.floor(p / cell).astype(int))
            ok = True
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dz in (-1, 0, 1):
                        for q in grid.get((c[0] + dx, c[1] + dy, c[2] + dz), ()):
                            v = p - pts[q]
                            if v @ v < d2:
                                ok = False
                                break
                        if not ok:
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if ok:
                pts[k] = p
                grid.setdefault(c, []).append(k)
                break
        else:
            return None
    return pts


def random_solute(rng, n, side, probs, dmin=0.9) -> System:
    """Non-periodic cluster: species drawn with `probs`, RSA in a cube."""
    while True:
        pts = _rsa(rng, n, (0, 0, 0), (side, side, side), dmin)
        if pts is not None:
            break
    spec = rng.choice(len(probs), size=n, p=probs).astype(np.int32)
    return System(pts.astype(np.float32), spec, np.zeros(3, np.float32))


def config0(seed: int = 0) -> System:
    """24 atoms, species uniform over H/C/N/O, uniform in an 8 A cube with
    rejection of pairs closer than 0.9 A; non-periodic."""
    rng = np.random.default_rng(seed)
    pts = None
    while pts is None:
        pts = _rsa(rng, 24, (0, 0, 0), (8.0, 8.0, 8.0), 0.9)
    spec = rng.integers(0, 4, size=24).astype(np.int32)
    return System(pts.astype(np.float32), spec, np.zeros(3, np.float32))


def _random_rotations(rng, k):
    """Uniform random rotation matrices from unit quaternions."""
    q = rng.normal(size=(k, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((k, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _water_molecules(rng, sites, jitter=0.05):
    """O at each site, two H at 0.96 A with a 104.5 deg angle, random
    orientation, then Gaussian jitter on every atom.  Order: O, H, H."""
    k = len(sites)
    ang = math.radians(HOH_ANGLE_DEG)
    local = np.array([[0.0, 0.0, 0.0],
                      [OH_BOND, 0.0, 0.0],
                      [OH_BOND * math.cos(ang), OH_BOND * math.sin(ang), 0.0]])
    R = _random_rotations(rng, k)
    pos = sites[:, None, :] + np.einsum("kij,aj->kai", R, local)
    pos = pos + rng.normal(0.0, jitter, size=pos.shape)
    spec = np.tile(np.array([O, H, H], np.int32), k)
    return pos.reshape(-1, 3), spec


def water_box(n_mol: int, seed: int, jitter: float = 0.05) -> System:
    """Periodic cubic water box at 1 g/cm^3; molecules on a jittered simple
    cubic lattice (random subset of sites), coordinates wrapped to [0, L)."""
    rng = np.random.default_rng(seed)
    L = (n_mol * WATER_VOL_A3) ** (1.0 / 3.0)
    n_side = max(1, int(math.ceil(n_mol ** (1.0 / 3.0))))
    a = L / n_side
    g = (np.arange(n_side) + 0.5) * a
    sites = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pick = rng.choice(len(sites), size=n_mol, replace=False)
    pos, spec = _water_molecules(rng, sites[np.sort(pick)], jitter)
    box = np.array([L, L, L])
    pos = pos - np.floor(pos / box) * box
    pos32 = pos.astype(np.float32)
    box32 = box.astype(np.float32)
    # float32 rounding can land exactly on L; keep every coordinate in [0, L)
    pos32 = np.where(pos32 >= box32, pos32 - box32, pos32).astype(np.float32)
    pos32 = np.where(pos32 < 0, 0.0, pos32).astype(np.float32)
    return System(pos32, spec, box32)


def config1(seed: int = 1) -> System:
    """Periodic water box: 667 molecules = 2,001 atoms (H:O = 2:1), L = 27.12 A."""
    return water_box(667, seed)


CONFIG2_PROBS = np.array([0.45, 0.30, 0.08, 0.10, 0.02, 0.03, 0.02])  # H C N O S F Cl


def ragged_solutes(n_systems: int, seed: int, nmin=10, nmax=120) -> Batch:
    """Independent non-periodic solutes with n ~ U{nmin..nmax}, species
    H/C/N/O/F/S/Cl at 0.45/0.30/0.08/0.10/0.03/0.02/0.02, RSA positions in a
    cube of side 1.2 A * n^(1/3) with 0.9 A rejection."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(nmin, nmax + 1, size=n_systems)
    systems = [random_solute(rng, int(n), 1.2 * float(n) ** (1.0 / 3.0), CONFIG2_PROBS)
               for n in sizes]
    return make_batch(systems)


def config2(seed: int = 2) -> Batch:
    return ragged_solutes(512, seed)


PROTEIN_PROBS = np.array([0.50, 0.315, 0.087, 0.095, 0.003, 0.0, 0.0])


def solvated_protein(seed: int = 3, n_protein: int = 30000, n_water_mol: int = 23334,
                     protein_density: float = 0.11) -> System:
    """Periodic cubic box: a protein-like sphere of RSA atoms (H/C/N/O/S at an
    average amino-acid composition) surrounded by lattice water at 1 g/cm^3,
    kept outside the sphere radius + 1 A."""
    rng = np.random.default_rng(seed)
    R = (3.0 * n_protein / (4.0 * math.pi * protein_density)) ** (1.0 / 3.0)
    a0 = WATER_VOL_A3 ** (1.0 / 3.0)
    L = ((4.0 / 3.0) * math.pi * (R + 1.0) ** 3 + n_water_mol * WATER_VOL_A3) ** (1.0 / 3.0)
    while True:
        n_side = int(round(L / a0))
        a = L / n_side
        g = (np.arange(n_side) + 0.5) * a
        sites = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
        r = np.linalg.norm(sites - L / 2, axis=1)
        free = sites[r > R + 1.0 + 0.5 * a]
        if len(free) >= n_water_mol:
            break
        L *= 1.005
    centre = np.full(3, L / 2)
    inside = lambda p: np.sum((p - centre) ** 2) < R * R
    prot = _rsa(rng, n_protein, centre - R, centre + R, 0.9, inside=inside, max_tries=100000)
    assert prot is not None
    pspec = rng.choice(7, size=n_protein, p=PROTEIN_PROBS / PROTEIN_PROBS.sum()).astype(np.int32)
    pick = np.sort(rng.choice(len(free), size=n_water_mol, replace=False))
    wpos, wspec = _water_molecules(rng, free[pick])
    pos = np.concatenate([prot, wpos])
    spec = np.concatenate([pspec, wspec])
    box = np.array([L, L, L])
    pos = pos - np.floor(pos / box) * box
    pos32 = pos.astype(np.float32)
    box32 = box.astype(np.float32)
    pos32 = np.where(pos32 >= box32, pos32 - box32, pos32).astype(np.float32)
    return System(pos32, spec.astype(np.int32), box32)


def config3(seed: int = 3) -> System:
    """~100,000-atom periodic solvated-protein-like box (~100 A)."""
    return solvated_protein(seed)


def perturb(coords: np.ndarray, rng, sigma: float = 0.01) -> np.ndarray:
    """One MD-like step: add N(0, sigma) to every coordinate (random walk)."""
    return (coords + rng.normal(0.0, sigma, size=coords.shape)).astype(np.float32)


@dataclass
class Request:
    arrival: float      # seconds from trace start
    system: System
    n_steps: int
    seed: int


def request_trace(n_requests: int, seed: int = 4, rate: float = 2000.0,
                  nmin: int = 20, nmax: int = 5000, n_steps: int = 50):
    """Poisson arrivals; sizes log-uniform in [nmin, nmax]; half periodic water
    boxes (3*round(n/3) atoms), half solutes built like the ragged batch."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    out = []
    for k in range(n_requests):
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        sub = int(rng.integers(0, 2**31 - 1))
        if rng.random() < 0.5:
            sys_ = water_box(max(1, int(round(n / 3))), sub)
        else:
            r2 = np.random.default_rng(sub)
            sys_ = random_solute(r2, n, 1.2 * float(n) ** (1.0 / 3.0), CONFIG2_PROBS)
        out.append(Request(arrival=float(t[k]), system=sys_, n_steps=n_steps, seed=sub))
    return out
