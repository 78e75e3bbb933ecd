"""Seeded synthetic inputs for the DMC hot path.

This module draws the inputs that both the HIP library and the CPU oracle
consume: ion geometry, contracted Cartesian Gaussian shells, LCAO
coefficients, Pade Jastrow parameters, initial walkers and (for the
multideterminant form) excitation lists with CI coefficients.  It performs
none of the method's arithmetic; it only fixes sizes, seeds and value
distributions.  The paper's molecules, basis sets and trial orbitals are
not available, so these stand in for them (QMC section: Slater-Jastrow
trial function of Eq. 2 built from LCAO orbitals phi_i = sum_l C_l^i Phi_l).

Seeding: every workload uses numpy.random.SeedSequence(250407948 + id),
spawned once per drawn object, so each object is reproducible on its own.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

BASE_SEED = 250407948

# number of Cartesian components per angular momentum (s, p, d)
NCART = (1, 3, 6)


@dataclasses.dataclass
class System:
    """One molecule: ions, basis, orbitals, Jastrow and optional CI expansion.

    Basis order is atom -> shell -> Cartesian component, with p = (x, y, z)
    and d = (xx, xy, xz, yy, yz, zz).  ``prim_coef`` already holds the
    primitive normalisation times the contraction coefficient, so both
    implementations evaluate R(r) = sum_p prim_coef[p] exp(-alpha_p r^2).
    ``mo_coef`` is [n_basis, n_mo] row-major; the up determinant uses MOs
    0..n_up-1 and the down determinant MOs 0..n_dn-1 (restricted orbitals).
    """

    name: str
    ion_xyz: np.ndarray          # [n_atom, 3] f64 (bohr)
    ion_charge: np.ndarray       # [n_atom] f64 (effective charge)
    shell_atom: np.ndarray       # [n_shell] i32
    shell_l: np.ndarray          # [n_shell] i32 in {0,1,2}
    shell_nprim: np.ndarray      # [n_shell] i32
    prim_alpha: np.ndarray       # [n_prim] f64
    prim_coef: np.ndarray        # [n_prim] f64
    mo_coef: np.ndarray          # [n_basis, n_mo] f64
    n_up: int
    n_dn: int
    jee_a_anti: float = 0.5
    jee_a_para: float = 0.25
    jee_b: float = 1.0
    jen_a: Optional[np.ndarray] = None   # [n_atom] f64, default -Z (cusp)
    jen_b: float = 0.8
    # multideterminant expansion (n_det == 0 -> single determinant)
    n_det: int = 0
    active_mo: Optional[np.ndarray] = None   # [n_active] i32, MO index
    det_exc: Optional[np.ndarray] = None     # [n_det, 8] i32 (see make_msd)
    ci_coef: Optional[np.ndarray] = None     # [n_det] f64
    # semilocal pseudopotential terms beta r^(n-2) exp(-alpha r^2): atom,
    # channel l (-1 local, >= 0 non-local), n, beta, alpha; rcut per atom
    pp_atom: Optional[np.ndarray] = None     # [n_term] i32
    pp_l: Optional[np.ndarray] = None        # [n_term] i32
    pp_n: Optional[np.ndarray] = None        # [n_term] i32
    pp_beta: Optional[np.ndarray] = None     # [n_term] f64
    pp_alpha: Optional[np.ndarray] = None    # [n_term] f64
    pp_rcut: Optional[np.ndarray] = None     # [n_atom] f64

    def __post_init__(self):
        self.ion_xyz = np.ascontiguousarray(self.ion_xyz, dtype=np.float64)
        self.ion_charge = np.ascontiguousarray(self.ion_charge, dtype=np.float64)
        self.shell_atom = np.ascontiguousarray(self.shell_atom, dtype=np.int32)
        self.shell_l = np.ascontiguousarray(self.shell_l, dtype=np.int32)
        self.shell_nprim = np.ascontiguousarray(self.shell_nprim, dtype=np.int32)
        self.prim_alpha = np.ascontiguousarray(self.prim_alpha, dtype=np.float64)
        self.prim_coef = np.ascontiguousarray(self.prim_coef, dtype=np.float64)
        self.mo_coef = np.ascontiguousarray(self.mo_coef, dtype=np.float64)
        if self.jen_a is None:
            self.jen_a = -self.ion_charge.copy()
        self.jen_a = np.ascontiguousarray(self.jen_a, dtype=np.float64)

    @property
    def n_atom(self) -> int:
        return int(self.ion_xyz.shape[0])

    @property
    def n_shell(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def n_basis(self) -> int:
        return int(self.mo_coef.shape[0])

    @property
    def n_mo(self) -> int:
        return int(self.mo_coef.shape[1])

    @property
    def n_elec(self) -> int:
        return self.n_up + self.n_dn


def gto_norm(alpha: np.ndarray, l: int) -> np.ndarray:
    """Primitive normalisation (2a/pi)^(3/4) (4a)^(l/2), folded into prim_coef."""
    return (2.0 * alpha / math.pi) ** 0.75 * (4.0 * alpha) ** (0.5 * l)


def _place_ions(rng, n_atom, box, min_dist_fn, max_tries=200000):
    pos = []
    tries = 0
    while len(pos) < n_atom:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("ion placement did not converge")
        p = rng.uniform(0.0, box, size=3)
        k = len(pos)
        if all(np.linalg.norm(p - q) >= min_dist_fn(k, j) for j, q in enumerate(pos)):
            pos.append(p)
    return np.array(pos)


def _shells_for(rng, atoms_shells, alpha_lo, alpha_hi, nprim):
    """atoms_shells: list of lists of l values, one list per atom."""
    sa, sl, sn, al, co = [], [], [], [], []
    for a, ls in enumerate(atoms_shells):
        for l in ls:
            alpha = np.exp(rng.uniform(math.log(alpha_lo), math.log(alpha_hi), size=nprim))
            d = rng.uniform(0.5, 1.5, size=nprim)
            sa.append(a)
            sl.append(l)
            sn.append(nprim)
            al.extend(alpha.tolist())
            co.extend((d * gto_norm(alpha, l)).tolist())
    return (np.array(sa), np.array(sl), np.array(sn), np.array(al), np.array(co))


def _orthonormal_mos(rng, n_basis, n_mo):
    """First n_mo columns of Q from the QR of a seeded N(0,1) matrix, signs
    fixed so that diag(R) > 0 (the reduced QR gives the same columns)."""
    g = rng.standard_normal((n_basis, n_mo))
    q, r = np.linalg.qr(g)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :]


def small_molecule() -> System:
    """4 ions, Z=2, uniform in a 6 bohr box (min spacing 1.0), 8 e (4/4),
    per atom 4s + 2p single-primitive shells, alpha log-U[0.2, 20] (40
    functions), 4 MOs per spin; Pade b_ee = 1.0, b_en = 0.8."""
    ss = np.random.SeedSequence(BASE_SEED + 1)
    s_geo, s_bas, s_mo = [np.random.default_rng(s) for s in ss.spawn(3)]
    xyz = _place_ions(s_geo, 4, 6.0, lambda i, j: 1.0)
    z = np.full(4, 2.0)
    sa, sl, sn, al, co = _shells_for(s_bas, [[0, 0, 0, 0, 1, 1]] * 4, 0.2, 20.0, 1)
    nb = int(sum(NCART[l] for l in sl))
    mo = _orthonormal_mos(s_mo, nb, 4)
    return System("small-4ion-8e", xyz, z, sa, sl, sn, al, co, mo, 4, 4, jee_b=1.0, jen_b=0.8)


def molecule(name: str) -> System:
    """The two synthetic molecules by name: "small" (8 electrons, 40
    functions) or "large" (112 electrons, 1024 functions)."""
    if name == "small":
        return small_molecule()
    if name == "large":
        return large_molecule()
    raise ValueError(f"unknown molecule {name!r}")


# per-molecule offsets of the seeds the tests and benchmark draw walkers with
SEED_OFFSET = {"small": 1, "large": 2}


def large_molecule() -> System:
    """64 ions (16 "C" with Z_eff = 4, 48 H) in a 16 bohr cube, min spacing
    1.5 bohr C-C and 1.1 bohr otherwise, 112 e (56/56); "C" 4s4p2d, "H"
    3s1p1d, three primitives per shell, alpha log-U[0.05, 50] -> 400 shells,
    1200 primitives, 1024 Cartesian functions; 56 MOs per spin."""
    ss = np.random.SeedSequence(BASE_SEED + 2)
    s_geo, s_bas, s_mo = [np.random.default_rng(s) for s in ss.spawn(3)]
    n_c, n_h = 16, 48
    kind = np.array([0] * n_c + [1] * n_h)      # 0 = "C" (Z_eff 4), 1 = "H"

    def mind(i, j):
        return 1.5 if (kind[i] == 0 and kind[j] == 0) else 1.1

    xyz = _place_ions(s_geo, n_c + n_h, 16.0, mind)
    z = np.where(kind == 0, 4.0, 1.0)
    c_sh = [0] * 4 + [1] * 4 + [2] * 2
    h_sh = [0] * 3 + [1] + [2]
    sa, sl, sn, al, co = _shells_for(
        s_bas, [c_sh if k == 0 else h_sh for k in kind], 0.05, 50.0, 3)
    nb = int(sum(NCART[l] for l in sl))
    mo = _orthonormal_mos(s_mo, nb, 56)
    return System("large-64ion-112e", xyz, z, sa, sl, sn, al, co, mo, 56, 56, jee_b=1.0, jen_b=0.8)


def make_walkers(sys: System, n_walkers: int, seed: int, sigma: float = 0.6) -> np.ndarray:
    """Initial walkers [W, n_elec, 3]: each atom receives round(Z_A) electrons,
    spins alternate over the electron list (atom order), up electrons are
    stored first; each electron sits at R_A + N(0, sigma^2 I)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    home_up, home_dn = [], []
    k = 0
    for a in range(sys.n_atom):
        for _ in range(int(round(sys.ion_charge[a]))):
            (home_up if k % 2 == 0 else home_dn).append(a)
            k += 1
    # pad / trim so the counts match n_up / n_dn (synthetic charged cases)
    allh = home_up + home_dn
    while len(home_up) < sys.n_up:
        home_up.append(allh[len(home_up) % len(allh)])
    while len(home_dn) < sys.n_dn:
        home_dn.append(allh[len(home_dn) % len(allh)])
    homes = np.array(home_up[: sys.n_up] + home_dn[: sys.n_dn], dtype=np.int64)
    centers = sys.ion_xyz[homes]
    R = centers[None, :, :] + sigma * rng.standard_normal((n_walkers, sys.n_elec, 3))
    return np.ascontiguousarray(R)


def small_random_system(seed: int, n_atom: int = 2, n_up: int = 2, n_dn: int = 2,
                        shells=(0, 0, 1, 2), nprim: int = 2, n_mo: Optional[int] = None,
                        box: float = 3.0, alpha=(0.3, 3.0), charge: float = 2.0) -> System:
    """Tiny systems for pins and edge cases (all shell types, contractions)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    xyz = _place_ions(rng, n_atom, box, lambda i, j: 0.8)
    z = np.full(n_atom, charge)
    sa, sl, sn, al, co = _shells_for(rng, [list(shells)] * n_atom, alpha[0], alpha[1], nprim)
    nb = int(sum(NCART[l] for l in sl))
    n_mo = max(n_up, n_dn) if n_mo is None else n_mo
    mo = _orthonormal_mos(rng, nb, n_mo)
    return System(f"small{seed}", xyz, z, sa, sl, sn, al, co, mo, n_up, n_dn)


# ------------------------------------------------------------------ MSD ----
def make_msd(sys: System, n_det: int, n_active: int, seed: int,
             frac_single: float = 0.1) -> System:
    """Attach a multideterminant expansion (Eq. 2 with M > 1).

    Active space: the last min(n_occ, n_active//2) occupied MOs plus the
    following virtuals, n_active in total; the MO matrix is extended with
    extra seeded orthonormal columns when needed.  Determinant 0 is the
    reference (c_0 = 1).  Each further determinant is a distinct single or
    double excitation drawn uniformly: a fraction ``frac_single`` singles,
    the rest split evenly over up-up, down-down and up-down doubles; the
    r-th draw gets |c_r| = exp(-0.01 r) with a random sign.

    det_exc[d] = [n_exc_up, n_exc_dn, hole_up0, part_up0, hole_up1/hole_dn0 ...]
    laid out as (nu, nd, h_u[0], h_u[1], p_u[0], p_u[1], h_d[0]... ) packed
    into 10 slots: [nu, nd, hu0, hu1, pu0, pu1, hd0, hd1, pd0, pd1] with
    holes as occupied-orbital indices and particles as MO indices (>= n_occ
    of that spin); unused slots are -1.
    """
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    n_occ = max(sys.n_up, sys.n_dn)
    n_occ_act = min(n_occ, n_active // 2)
    n_virt = n_active - n_occ_act
    need_mo = n_occ + n_virt
    mo = sys.mo_coef
    if mo.shape[1] < need_mo:
        extra = rng.standard_normal((mo.shape[0], need_mo - mo.shape[1]))
        full = np.concatenate([mo, extra], axis=1)
        q, r = np.linalg.qr(full)
        s = np.sign(np.diag(r))
        s[s == 0] = 1.0
        q = q * s[None, :]
        # keep the original columns exactly
        mo = np.concatenate([mo, q[:, mo.shape[1]:]], axis=1)
    active = np.array(list(range(n_occ - n_occ_act, n_occ)) +
                      list(range(n_occ, n_occ + n_virt)), dtype=np.int32)
    occ_up = list(range(sys.n_up - min(sys.n_up, n_occ_act), sys.n_up))
    occ_dn = list(range(sys.n_dn - min(sys.n_dn, n_occ_act), sys.n_dn))
    virt = list(range(n_occ, n_occ + n_virt))
    seen = set()
    exc = [[0, 0] + [-1] * 8]
    kinds = []
    n_single = int(round(frac_single * (n_det - 1)))
    n_double = n_det - 1 - n_single
    kinds += ["s"] * n_single
    kinds += [("uu", "dd", "ud")[i % 3] for i in range(n_double)]
    rng.shuffle(kinds)
    for kd in kinds:
        for _ in range(10000):
            if kd == "s":
                spin = rng.integers(2)
                occ = occ_up if spin == 0 else occ_dn
                h = [int(rng.choice(occ))]
                p = [int(rng.choice(virt))]
                key = (kd, spin, tuple(h), tuple(p))
                row = ([1, 0, h[0], -1, p[0], -1, -1, -1, -1, -1] if spin == 0 else
                       [0, 1, -1, -1, -1, -1, h[0], -1, p[0], -1])
            elif kd in ("uu", "dd"):
                occ = occ_up if kd == "uu" else occ_dn
                h = sorted(rng.choice(occ, 2, replace=False).tolist())
                p = sorted(rng.choice(virt, 2, replace=False).tolist())
                key = (kd, tuple(h), tuple(p))
                row = ([2, 0, h[0], h[1], p[0], p[1], -1, -1, -1, -1] if kd == "uu" else
                       [0, 2, -1, -1, -1, -1, h[0], h[1], p[0], p[1]])
            else:
                hu, hd = int(rng.choice(occ_up)), int(rng.choice(occ_dn))
                pu, pd = int(rng.choice(virt)), int(rng.choice(virt))
                key = (kd, hu, hd, pu, pd)
                row = [1, 1, hu, -1, pu, -1, hd, -1, pd, -1]
            if key not in seen:
                seen.add(key)
                exc.append(row)
                break
        else:
            raise RuntimeError("could not draw distinct excitations")
    ranks = np.arange(1, n_det)
    mag = np.exp(-0.01 * ranks)
    sign = np.where(rng.random(n_det - 1) < 0.5, -1.0, 1.0)
    ci = np.concatenate([[1.0], mag * sign])
    out = dataclasses.replace(sys)
    out.mo_coef = np.ascontiguousarray(mo)
    out.n_det = n_det
    out.active_mo = active
    out.det_exc = np.ascontiguousarray(np.array(exc, dtype=np.int32))
    out.ci_coef = np.ascontiguousarray(ci)
    return out


def alkane(n_c: int, seed: int) -> System:
    """C_nH_(2n+2) stand-in: a zig-zag carbon chain (1.54 bohr-scaled steps)
    with hydrogens placed around it; Z_eff = 4 for C, basis as in the large molecule."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    bond = 2.9  # bohr
    cpos = []
    for i in range(n_c):
        cpos.append([i * bond * 0.82, (i % 2) * bond * 0.57, 0.0])
    cpos = np.array(cpos)
    hpos = []
    for i in range(n_c):
        nh = 3 if i in (0, n_c - 1) else 2
        if n_c == 1:
            nh = 4
        for k in range(nh):
            d = rng.standard_normal(3)
            d /= np.linalg.norm(d)
            hpos.append(cpos[i] + 2.06 * d)
    xyz = np.concatenate([cpos, np.array(hpos)], axis=0)
    kind = np.array([0] * n_c + [1] * len(hpos))
    z = np.where(kind == 0, 4.0, 1.0)
    c_sh = [0] * 4 + [1] * 4 + [2] * 2
    h_sh = [0] * 3 + [1] + [2]
    sa, sl, sn, al, co = _shells_for(
        rng, [c_sh if k == 0 else h_sh for k in kind], 0.05, 50.0, 3)
    nb = int(sum(NCART[l] for l in sl))
    ne = int(round(z.sum()))
    nup = ne // 2
    mo = _orthonormal_mos(rng, nb, nup)
    return System(f"C{n_c}H{2*n_c+2}", xyz, z, sa, sl, sn, al, co, mo, nup, ne - nup)


ALKANE_NC = (3, 7, 11, 16, 20, 24, 29, 33)


def batch5_member(k: int, n_det: int = 1000, n_active: int = 100) -> System:
    """Molecule k (0..7) of the eight-alkane workload, with its MSD expansion."""
    s = alkane(ALKANE_NC[k], BASE_SEED + 5 + 1000 * k)
    return make_msd(s, n_det, n_active, BASE_SEED + 5 + 1000 * k + 1)


def make_batch5(n_det: int = 1000, n_active: int = 100) -> List[System]:
    """Eight alkanes with 20..200 electrons, each with an MSD expansion."""
    return [batch5_member(k, n_det, n_active) for k in range(len(ALKANE_NC))]


# ------------------------------------------------------- pseudopotentials ----
def pp_rcut_for(terms, eps: float = 1e-16) -> float:
    """Radius beyond which every non-local term |beta| r^(n-2) exp(-alpha r^2)
    of an atom is below eps |beta| (n = 2 terms: sqrt(ln(1/eps) / alpha))."""
    r = 0.0
    for l, n, beta, alpha in terms:
        if l < 0:
            continue
        rr = np.sqrt(np.log(1.0 / eps) / alpha)
        # a power r^(n-2) > 1 pushes the radius out a little
        while n > 2 and rr ** (n - 2) * np.exp(-alpha * rr * rr) > eps:
            rr *= 1.05
        r = max(r, rr)
    return float(r)


def with_pseudopotential(sys: System, terms_by_atom) -> System:
    """A copy of sys with semilocal pseudopotential terms: terms_by_atom[A] is
    a list of (l, n, beta, alpha), l = -1 local, l >= 0 non-local; atoms with
    an empty list keep the bare Coulomb potential."""
    import dataclasses
    at, ll, nn, bb, aa = [], [], [], [], []
    rcut = np.zeros(sys.n_atom)
    for A, terms in enumerate(terms_by_atom):
        for l, n, beta, alpha in terms:
            at.append(A)
            ll.append(l)
            nn.append(n)
            bb.append(beta)
            aa.append(alpha)
        rcut[A] = pp_rcut_for(terms)
    return dataclasses.replace(
        sys, name=sys.name + "-pp", pp_atom=np.array(at, np.int32), pp_l=np.array(ll, np.int32),
        pp_n=np.array(nn, np.int32), pp_beta=np.array(bb, np.float64),
        pp_alpha=np.array(aa, np.float64), pp_rcut=rcut)


# Synthetic stand-ins for the ccECP tables (not available here), in the same
# functional form: for the Z_eff = 2 atoms of the small molecule a local term
# and non-local s and p channels; for the "C" (Z_eff = 4) atoms of the large
# molecule a local term and a non-local s channel, the H atoms all-electron.
PP_SMALL = [(-1, 2, -2.5, 2.0), (0, 2, 3.0, 2.5), (1, 2, -1.0, 2.0)]
PP_CARBON = [(-1, 2, -5.0, 3.0), (0, 2, 6.0, 8.0)]


def small_molecule_pp() -> System:
    """The small molecule with PP_SMALL on every atom."""
    s = small_molecule()
    return with_pseudopotential(s, [PP_SMALL] * s.n_atom)


def large_molecule_pp() -> System:
    """The large molecule with PP_CARBON on its 16 "C" atoms."""
    s = large_molecule()
    return with_pseudopotential(s, [PP_CARBON if z == 4.0 else [] for z in s.ion_charge])
