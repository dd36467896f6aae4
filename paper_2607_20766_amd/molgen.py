"""Seeded synthetic molecules: the only input source shared by the HIP path and
the CPU oracle.

This module builds geometry and nothing else.  It holds none of the
estimator's arithmetic: no Gaussian widths, no densities, no sampling weights.
Both sides derive everything else (atom Gaussian widths from the radii, mixture
weights, sample points) on their own.

Molecules are random branched heavy-atom chains standing in for drug-like
ligands (the paper's panel uses drug-like molecules embedded with RDKit, which
is not available here):

* bond length 1.50 A, bond angle uniform in [104.5, 114.5] degrees
  (109.5 +- 5), torsion uniform in [-pi, pi);
* growth: with probability 0.75 the newest atom is extended (if it has fewer
  than four bonds), otherwise a uniformly random atom with fewer than four
  bonds receives the new atom;
* a candidate is accepted when every angle it makes with the parent's existing
  bonds is at least 100 degrees and every atom three or more bonds away lies at
  least 2.5 A from it; after 50 rejected torsion/angle draws a new parent is
  chosen uniformly among atoms with free valence;
* element types are drawn i.i.d.: C/N/O/S with p = 0.70/0.15/0.12/0.03 and van
  der Waals radii 1.70/1.55/1.52/1.80 A.

Every molecule is then centred and rotated into its principal inertial frame,
weighting each atom by R^3 (its hard-sphere volume up to a constant).  Axes
are sorted by decreasing second moment; the first two are oriented so that the
third moment of the atom projections is non-negative and the third axis is
their cross product, giving a proper rotation.

Molecules are generated in vectorised batches.  A batch is fully determined by
``numpy.random.SeedSequence(entropy)``; a library of M molecules is split into
chunks of ``CHUNK`` molecules, chunk c using entropy ``[config_seed, 0x11B, c]``
and the atom counts using ``[config_seed, 0x512E]``.  A single molecule
(``molecule(config_seed, index, n)``) uses entropy ``[config_seed, index]``.
"""
from __future__ import annotations

import concurrent.futures
import dataclasses
import math
import multiprocessing
import os

import numpy as np

ELEMENTS = ("C", "N", "O", "S")
ELEMENT_P = np.array([0.70, 0.15, 0.12, 0.03])
VDW_RADIUS = np.array([1.70, 1.55, 1.52, 1.80])

BOND = 1.50
ANGLE_LO = math.radians(104.5)
ANGLE_HI = math.radians(114.5)
MIN_BOND_ANGLE = math.radians(100.0)
NONBONDED_MIN = 2.5
TORSION_TRIES = 50
KBATCH = 10
CHUNK = 16384


@dataclasses.dataclass
class MolSet:
    """A set of molecules in CSR layout (host arrays).

    offsets: int32 [n_mols + 1]; atoms of molecule m are offsets[m]:offsets[m+1]
    xyz:     float32 [n_atoms, 3] in Angstrom, each molecule in its own frame
    radius:  float32 [n_atoms] van der Waals radius in Angstrom
    element: int8 [n_atoms] index into ELEMENTS
    """

    offsets: np.ndarray
    xyz: np.ndarray
    radius: np.ndarray
    element: np.ndarray

    @property
    def n_mols(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_atoms(self) -> int:
        return int(self.offsets[-1])

    def sizes(self) -> np.ndarray:
        return np.diff(self.offsets)

    def mol(self, m: int) -> "MolSet":
        a, b = int(self.offsets[m]), int(self.offsets[m + 1])
        return MolSet(np.array([0, b - a], np.int32), self.xyz[a:b].copy(),
                      self.radius[a:b].copy(), self.element[a:b].copy())

    def subset(self, idx) -> "MolSet":
        idx = np.asarray(idx, dtype=np.int64)
        sz = self.sizes()[idx]
        off = np.zeros(idx.size + 1, np.int64)
        np.cumsum(sz, out=off[1:])
        sel = np.concatenate([np.arange(self.offsets[m], self.offsets[m + 1])
                              for m in idx]) if idx.size else np.zeros(0, np.int64)
        return MolSet(off.astype(np.int32), self.xyz[sel].copy(),
                      self.radius[sel].copy(), self.element[sel].copy())

    @staticmethod
    def concat(sets) -> "MolSet":
        sizes = np.concatenate([s.sizes() for s in sets])
        off = np.zeros(sizes.size + 1, np.int64)
        np.cumsum(sizes, out=off[1:])
        return MolSet(off.astype(np.int32),
                      np.concatenate([s.xyz for s in sets]),
                      np.concatenate([s.radius for s in sets]),
                      np.concatenate([s.element for s in sets]))


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _random_perp(rng, u):
    """A random unit vector perpendicular to each row of u."""
    while True:
        g = rng.standard_normal(u.shape)
        g -= (g * u).sum(-1, keepdims=True) * u
        n = np.linalg.norm(g, axis=-1, keepdims=True)
        if np.all(n > 1e-6):
            return g / n


def _grow_batch(rng: np.random.Generator, sizes: np.ndarray, fixed_parents=None,
                parents_out=None):
    """Grow len(sizes) chains at once; returns positions [M, max(sizes), 3].

    fixed_parents [M, nmax] (optional) fixes the bonded parent of every atom,
    so the chains keep a given topology and only bond angles and torsions
    are redrawn (conformers); a chain whose atom finds no acceptable
    placement in 300 draws is abandoned and flagged in the second return
    value.  parents_out [M, nmax] (optional) receives the parents chosen.
    """
    M = sizes.size
    nmax = int(sizes.max())
    pos = np.zeros((M, nmax, 3))
    nbr = np.full((M, nmax, 4), -1, np.int32)
    deg = np.zeros((M, nmax), np.int32)
    topo = np.zeros((M, nmax, nmax), np.int16)
    failed = np.zeros(M, bool)

    def done():
        return pos if fixed_parents is None else (pos, failed)

    if nmax == 1:
        return done()
    # atom 1: random direction from atom 0
    act = np.nonzero(sizes > 1)[0]
    d = _unit(rng.standard_normal((act.size, 3)))
    pos[act, 1] = BOND * d
    nbr[act, 0, 0] = 1
    nbr[act, 1, 0] = 0
    deg[act, 0] = 1
    deg[act, 1] = 1
    topo[act, 0, 1] = topo[act, 1, 0] = 1

    if parents_out is not None:
        parents_out[:, :2] = [-1, 0]
    for t in range(2, nmax):
        act = np.nonzero((sizes > t) & ~failed)[0]

        def pick_random_parent(idx):
            free = deg[idx, :t] < 4
            r = rng.random((idx.size, t)) * free
            return np.argmax(r, axis=1).astype(np.int32)

        if fixed_parents is None:
            # parent choice
            newest_ok = deg[act, t - 1] < 4
            extend = (rng.random(act.size) < 0.75) & newest_ok
            parent = np.where(extend, t - 1, 0).astype(np.int32)
            nr = ~extend
            if nr.any():
                parent[nr] = pick_random_parent(act[nr])
        else:
            parent = fixed_parents[act, t].astype(np.int32)
        restarts = np.zeros(act.size, np.int32)
        tries = np.zeros(act.size, np.int32)
        todo = np.arange(act.size)
        guard = 0
        while todo.size:
            guard += 1
            if guard > 100000:
                raise RuntimeError("molecule growth did not terminate")
            mi = act[todo]
            p = parent[todo]
            ppos = pos[mi, p]
            # reference neighbour a: the parent's lowest-index neighbour
            a = nbr[mi, p, 0]
            u = _unit(pos[mi, a] - ppos)
            # dihedral reference b: a neighbour of a other than p
            na = nbr[mi, a]  # [k, 4]
            cand = np.where((na >= 0) & (na != p[:, None]), na, nmax + 1)
            b = cand.min(axis=1)
            has_b = b <= nmax
            v = np.empty_like(u)
            if has_b.any():
                bb = b[has_b]
                vb = pos[mi[has_b], bb] - pos[mi[has_b], a[has_b]]
                vb -= (vb * u[has_b]).sum(-1, keepdims=True) * u[has_b]
                nb = np.linalg.norm(vb, axis=-1, keepdims=True)
                ok = nb[:, 0] > 1e-6
                vv = np.empty_like(vb)
                vv[ok] = vb[ok] / nb[ok]
                if (~ok).any():
                    vv[~ok] = _random_perp(rng, u[has_b][~ok])
                v[has_b] = vv
            if (~has_b).any():
                v[~has_b] = _random_perp(rng, u[~has_b])
            w = np.cross(u, v)
            # K consecutive draws per molecule are evaluated at once; the first
            # acceptable one (in draw order) is taken, as if drawn one by one.
            K = 1 if todo.size > 512 else (KBATCH if fixed_parents is None else 5 * KBATCH)
            theta = rng.uniform(ANGLE_LO, ANGLE_HI, (todo.size, K))
            phi = rng.uniform(-math.pi, math.pi, (todo.size, K))
            dvec = (np.cos(theta)[..., None] * u[:, None] + np.sin(theta)[..., None]
                    * (np.cos(phi)[..., None] * v[:, None]
                       + np.sin(phi)[..., None] * w[:, None]))  # [k, K, 3]
            newp = ppos[:, None] + BOND * dvec
            # (i) angles with every existing bond of the parent
            nbp = nbr[mi, p]  # [k, 4]
            okang = np.ones((todo.size, K), bool)
            cmax = math.cos(MIN_BOND_ANGLE)
            for s in range(4):
                has = nbp[:, s] >= 0
                if has.any():
                    e = _unit(pos[mi[has], nbp[has, s]] - ppos[has])
                    okang[has] &= (e[:, None] * dvec[has]).sum(-1) <= cmax + 1e-12
            # (ii) non-bonded distances to atoms >= 3 bonds away
            dist2 = ((pos[mi, None, :t] - newp[:, :, None, :]) ** 2).sum(-1)
            far = topo[mi, p, :t] >= 2
            okd = ~np.any(far[:, None] & (dist2 < NONBONDED_MIN ** 2), axis=2)
            okk = okang & okd
            allowed = np.arange(K)[None, :] < (TORSION_TRIES - tries[todo])[:, None]
            okk &= allowed
            ok = okk.any(axis=1)
            first = np.argmax(okk, axis=1)
            # accept
            acc = todo[ok]
            if acc.size:
                am = act[acc]
                ap = parent[acc]
                pos[am, t] = newp[ok, first[ok]]
                slot = deg[am, ap]
                nbr[am, ap, slot] = t
                nbr[am, t, 0] = ap
                deg[am, ap] += 1
                deg[am, t] = 1
                topo[am, t, :t] = topo[am, ap, :t] + 1
                topo[am, :t, t] = topo[am, t, :t]
                if parents_out is not None:
                    parents_out[am, t] = ap
            rej = todo[~ok]
            tries[rej] = np.minimum(tries[rej] + K, TORSION_TRIES)
            re = rej[tries[rej] >= TORSION_TRIES]
            if re.size:
                tries[re] = 0
                if fixed_parents is None:
                    parent[re] = pick_random_parent(act[re])
                else:
                    restarts[re] += 1
                    dead = re[restarts[re] >= 6]
                    if dead.size:
                        failed[act[dead]] = True
                        rej = np.setdiff1d(rej, dead)
            todo = rej
    return done()


def principal_frame(xyz: np.ndarray, radius: np.ndarray) -> np.ndarray:
    """Centre on the R^3-weighted centroid and rotate into the principal frame."""
    w = radius.astype(np.float64) ** 3
    w = w / w.sum()
    c = xyz - (w[:, None] * xyz).sum(0)
    cov = (w[:, None, None] * c[:, :, None] * c[:, None, :]).sum(0)
    ev, evec = np.linalg.eigh(cov)
    order = np.argsort(ev)[::-1]
    e = evec[:, order].T.copy()  # rows = axes
    for k in range(2):
        if (w * (c @ e[k]) ** 3).sum() < 0:
            e[k] = -e[k]
    e[2] = np.cross(e[0], e[1])
    return c @ e.T


def principal_frame_batch(pos: np.ndarray, radius: np.ndarray) -> np.ndarray:
    """principal_frame over a padded batch [M, n, 3]; padding has radius 0."""
    w = radius.astype(np.float64) ** 3
    w = w / w.sum(1, keepdims=True)
    c = pos - (w[..., None] * pos).sum(1, keepdims=True)
    cov = np.einsum("mi,mia,mib->mab", w, c, c)
    ev, evec = np.linalg.eigh(cov)
    e = np.swapaxes(evec[:, :, ::-1], 1, 2).copy()  # rows = axes, descending
    for k in range(2):
        m3 = (w * np.einsum("mia,ma->mi", c, e[:, k]) ** 3).sum(1)
        e[m3 < 0, k] *= -1.0
    e[:, 2] = np.cross(e[:, 0], e[:, 1])
    return np.einsum("mia,mba->mib", c, e)


def _batch(entropy, sizes: np.ndarray) -> MolSet:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(entropy)))
    sizes = np.asarray(sizes, np.int64)
    pos = _grow_batch(rng, sizes)
    elem = rng.choice(len(ELEMENTS), size=(sizes.size, pos.shape[1]), p=ELEMENT_P)
    off = np.zeros(sizes.size + 1, np.int64)
    np.cumsum(sizes, out=off[1:])
    nmax = pos.shape[1]
    mask = np.arange(nmax)[None, :] < sizes[:, None]
    rad_pad = VDW_RADIUS[elem] * mask
    frame = principal_frame_batch(pos, rad_pad)
    xyz = frame[mask].astype(np.float32)
    el = elem[mask].astype(np.int8)
    rad = VDW_RADIUS[el].astype(np.float32)
    return MolSet(off.astype(np.int32), xyz, rad, el)


def molecule(config_seed: int, index: int, n_atoms: int) -> MolSet:
    """One molecule of n_atoms heavy atoms, seeded by (config_seed, index)."""
    if n_atoms < 1:
        raise ValueError("n_atoms must be >= 1")
    return _batch([int(config_seed), int(index)], np.array([n_atoms]))


def library_sizes(config_seed: int, n_mols: int, lo: int, hi: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(
        np.random.SeedSequence([int(config_seed), 0x512E])))
    return rng.integers(lo, hi + 1, size=n_mols)


def library(config_seed: int, n_mols: int, lo: int, hi: int,
            chunks=None, workers=None) -> MolSet:
    """n_mols molecules with atom counts uniform in [lo, hi].

    ``chunks`` optionally restricts generation to the listed chunk indices
    (each CHUNK molecules); the molecules produced are identical to those of
    the full library.
    """
    sizes = library_sizes(config_seed, n_mols, lo, hi)
    nch = (n_mols + CHUNK - 1) // CHUNK
    sel = list(range(nch) if chunks is None else chunks)
    jobs = [([int(config_seed), 0x11B, int(c)], sizes[c * CHUNK:(c + 1) * CHUNK])
            for c in sel]
    if workers is None:
        workers = min(len(jobs), 8, os.cpu_count() or 1)
    if workers > 1 and len(jobs) > 1:
        ctx = multiprocessing.get_context("fork")
        with concurrent.futures.ProcessPoolExecutor(workers, mp_context=ctx) as ex:
            parts = list(ex.map(_batch, *zip(*jobs)))
    else:
        parts = [_batch(e, s) for e, s in jobs]
    return MolSet.concat(parts)


CONF_CHUNK = 1024


def _conformer_chunk(config_seed: int, chunk: int, sizes: np.ndarray, n_conf: int):
    nm = sizes.size
    nmax = int(sizes.max())
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(
        [int(config_seed), 0xC0F, int(chunk)])))
    par = np.full((nm, nmax), -1, np.int32)
    base = _grow_batch(rng, sizes, parents_out=par)
    elem = rng.choice(len(ELEMENTS), size=(nm, nmax), p=ELEMENT_P)
    confs = [base]
    for c in range(1, n_conf):
        pos = np.zeros_like(base)
        todo = np.arange(nm)
        for attempt in range(20):
            r = np.random.Generator(np.random.PCG64(np.random.SeedSequence(
                [int(config_seed), 0xC0F, int(chunk), c, attempt])))
            p, failed = _grow_batch(r, sizes[todo], fixed_parents=par[todo])
            good = ~failed
            pos[todo[good], :p.shape[1]] = p[good]
            todo = todo[failed]
            if todo.size == 0:
                break
        pos[todo] = base[todo]  # not completed in 20 attempts: the grown shape
        confs.append(pos)
    allpos = np.stack(confs, 1).reshape(nm * n_conf, nmax, 3)
    el_all = np.repeat(elem, n_conf, axis=0)
    sz_all = np.repeat(sizes, n_conf)
    mask = np.arange(nmax)[None, :] < sz_all[:, None]
    frame = principal_frame_batch(allpos, VDW_RADIUS[el_all] * mask)
    off = np.zeros(sz_all.size + 1, np.int64)
    np.cumsum(sz_all, out=off[1:])
    el = el_all[mask].astype(np.int8)
    return MolSet(off.astype(np.int32), frame[mask].astype(np.float32),
                  VDW_RADIUS[el].astype(np.float32), el)


def conformer_library(config_seed: int, n_mols: int, lo: int, hi: int, n_conf: int,
                      workers=None) -> tuple[MolSet, np.ndarray]:
    """n_mols molecules with n_conf conformers each (the conformer-ensemble
    workload: the paper's accuracy lever is the max over conformers).

    Molecules come in chunks of CONF_CHUNK; atom counts are U{lo..hi} from
    seed sequence [seed, 0xC0F5].  Conformer 0 is the molecule as grown
    ([seed, 0xC0F, chunk]); conformers 1.. keep its topology and elements and
    redraw every bond angle and torsion under the same acceptance rules
    ([seed, 0xC0F, chunk, c, attempt]; a chain that cannot be completed is
    redrawn with the next attempt).  Each conformer is put into its own
    principal frame.  Returns the set (molecule-major: entry m n_conf + c)
    and group offsets [n_mols + 1] (multiples of n_conf).
    """
    sizes = np.random.Generator(np.random.PCG64(np.random.SeedSequence(
        [int(config_seed), 0xC0F5]))).integers(lo, hi + 1, size=n_mols).astype(np.int64)
    nch = (n_mols + CONF_CHUNK - 1) // CONF_CHUNK
    jobs = [(int(config_seed), c, sizes[c * CONF_CHUNK:(c + 1) * CONF_CHUNK], int(n_conf))
            for c in range(nch)]
    if workers is None:
        workers = min(nch, 16, os.cpu_count() or 1)
    if workers > 1 and nch > 1:
        ctx = multiprocessing.get_context("fork")
        with concurrent.futures.ProcessPoolExecutor(workers, mp_context=ctx) as ex:
            parts = list(ex.map(_conformer_chunk, *zip(*jobs)))
    else:
        parts = [_conformer_chunk(*j) for j in jobs]
    return MolSet.concat(parts), np.arange(0, n_mols * n_conf + 1, n_conf, dtype=np.int32)


def random_poses(config_seed: int, n_pairs: int, n_starts: int,
                 t_sigma: float = 1.0) -> np.ndarray:
    """Start poses [n_pairs, n_starts, 7] = (qw, qx, qy, qz, tx, ty, tz).

    Quaternions are uniform on SO(3) (Shoemake's subgroup algorithm, 1992);
    translations are N(0, t_sigma^2) per axis.
    """
    rng = np.random.Generator(np.random.PCG64(
        np.random.SeedSequence([int(config_seed), 0x9053])))
    u1, u2, u3 = rng.random((3, n_pairs, n_starts))
    a = np.sqrt(1.0 - u1)
    b = np.sqrt(u1)
    q = np.stack([b * np.cos(2 * np.pi * u3), a * np.sin(2 * np.pi * u2),
                  a * np.cos(2 * np.pi * u2), b * np.sin(2 * np.pi * u3)], -1)
    t = rng.standard_normal((n_pairs, n_starts, 3)) * t_sigma
    return np.concatenate([q, t], -1).astype(np.float32)
