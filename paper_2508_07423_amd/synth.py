"""Seeded synthetic inputs: detector events and random network weights.

This module holds the workload recipe only (straight tracks through a stack of
pixel planes, noise hits, Xavier-initialised weights).  It contains none of the
track-finding arithmetic; both the HIP path and the FP64 oracle consume what it
produces.

Detector model (stand-in for the private LHCb simulation the thesis trains and
measures on, ch. 8 "Datasets"): planes perpendicular to the beam at fixed z,
straight tracks from a luminous region (the VELO sees straight lines because
the magnet field does not reach it, ch. 7 "VELO Tracking"), pseudorapidity
2 < eta < 5, theta = 2 atan(exp(-eta)) (ch. 3, pseudorapidity), a 98 % hit
efficiency, 12 um transverse smearing and 5 % noise hits.

Seeds: event ``i`` of workload ``c`` draws from
``numpy.random.SeedSequence([c, i])``; layer ``l`` of a random weight set
drawn with seed ``s`` uses ``SeedSequence([s, l])``.
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field, replace
from typing import Dict, List, Optional, Tuple

import numpy as np


@dataclass(frozen=True)
class Workload:
    """One workload: detector geometry, event recipe and network sizes."""

    cid: int                      # seed namespace of the events
    name: str
    n_events: int
    z_planes: Tuple[float, ...]
    acceptance: Optional[Tuple[float, float]]   # transverse annulus (mm) a hit must fall in
    noise_annulus: Tuple[float, float]
    tracks: Tuple[str, float]     # ("fixed", n) | ("poisson", lam) | ("mixed", lam)
    r_scale: float                # R_s: feature normalisation radius (mm)
    z_scale: float                # Z_s: feature normalisation |z| (mm)
    emb_hidden: int
    emb_layers: int               # hidden layers of the embedding MLP
    emb_dim: int
    radius: float
    k_max: int
    plane_window: int
    gnn_hidden: int
    gnn_steps: int
    threshold: float = 0.5
    weight_seed: int = 0
    vertex_sigma_xy: float = 0.05
    vertex_sigma_z: float = 50.0
    eta_range: Tuple[float, float] = (2.0, 5.0)
    hit_efficiency: float = 0.98
    smear_xy: float = 0.012
    noise_fraction: float = 0.05
    # hit order inside an event: "readout" = plane by plane, by azimuth within a
    # plane (the order a module-by-module detector readout delivers, as the
    # thesis's GPU framework stores its hits); "shuffled" = random
    hit_order: str = "readout"
    # conversion pairs (the thesis's motivation for the triplet stage, ch. 8
    # "Shared hits"): this fraction of the tracks gets a partner particle that
    # shares the parent's first `pair_shared` hits (the same hits: too close to
    # be resolved) and then leaves them at a small opening angle (rad)
    pair_fraction: float = 0.0
    pair_shared: Tuple[int, int] = (1, 3)
    pair_angle: Tuple[float, float] = (0.003, 0.01)

    @property
    def n_planes(self) -> int:
        return len(self.z_planes)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


_Z10 = tuple(float(z) for z in np.arange(10) * 50.0)
_Z26 = tuple(float(-290.0 + 41.6 * p) for p in range(26))

# Plain pipeline, one event: 10 planes 0..450 mm, 50 tracks, emb 3-64-64-8,
# radius 0.1, k 32, IN hidden 32, 4 steps.
C1 = Workload(cid=1, name="c1", n_events=1, z_planes=_Z10, acceptance=None,
              noise_annulus=(5.0, 40.0), tracks=("fixed", 50), r_scale=40.0,
              z_scale=450.0, emb_hidden=64, emb_layers=2, emb_dim=8, radius=0.1,
              k_max=32, plane_window=2, gnn_hidden=32, gnn_steps=4, weight_seed=101)
# Plain FP32 at full size: 1000 events, 26 planes -290..750 mm, Poisson(200)
# tracks, emb 3-128-128-12, radius 0.12, k 64, IN hidden 64, 8 steps.
C2 = Workload(cid=2, name="c2", n_events=1000, z_planes=_Z26, acceptance=(5.0, 60.0),
              noise_annulus=(5.0, 60.0), tracks=("poisson", 200.0), r_scale=60.0,
              z_scale=750.0, emb_hidden=128, emb_layers=2, emb_dim=12, radius=0.12,
              k_max=64, plane_window=2, gnn_hidden=64, gnn_steps=8, weight_seed=102)
# Batching: 10,000 uneven events (20..600 tracks) on the c2 geometry, c1 network.
C3 = Workload(cid=3, name="c3", n_events=10000, z_planes=_Z26, acceptance=(5.0, 60.0),
              noise_annulus=(5.0, 60.0), tracks=("mixed", 150.0), r_scale=60.0,
              z_scale=750.0, emb_hidden=64, emb_layers=2, emb_dim=8, radius=0.1,
              k_max=32, plane_window=2, gnn_hidden=32, gnn_steps=4, weight_seed=101)
# Precision: the c2 workload (BF16 / FP8 chosen at run time).
C4 = C2.with_(cid=4, name="c4")
# Learned prefilter: the c3 workload; training events use a disjoint seed space.
C5 = C3.with_(cid=5, name="c5")

# Triplet stage: the c3 workload with conversion pairs (a tenth of the tracks
# gets a partner that shares its first one to three hits).
C6 = C3.with_(cid=6, name="c6", pair_fraction=0.1)

WORKLOADS: Dict[str, Workload] = {w.name: w for w in (C1, C2, C3, C4, C5, C6)}


def _n_tracks(w: Workload, rng: np.random.Generator) -> int:
    kind, lam = w.tracks
    if kind == "fixed":
        return int(lam)
    if kind == "poisson":
        return int(rng.poisson(lam))
    # "mixed": a log-normal spread of the Poisson mean, so that event sizes
    # span the uneven 20..600-track range the batching workload asks for.
    z = rng.standard_normal()
    n = int(rng.poisson(lam * np.exp(0.8 * z - 0.32)))
    return int(min(max(n, 20), 600))


def generate_event(w: Workload, index: int, seed_space: Optional[int] = None) -> Dict[str, np.ndarray]:
    """One event as SoA arrays, hits in the workload's order (``hit_order``).

    Returns x, y, z (float32, mm), plane (int32), particle (int32, -1 = noise).
    """
    rng = np.random.default_rng(np.random.SeedSequence([w.cid if seed_space is None else seed_space, index]))
    zp = np.asarray(w.z_planes, dtype=np.float64)
    nt = _n_tracks(w, rng)
    vx = rng.normal(0.0, w.vertex_sigma_xy, nt)
    vy = rng.normal(0.0, w.vertex_sigma_xy, nt)
    vz = rng.normal(0.0, w.vertex_sigma_z, nt)
    eta = rng.uniform(w.eta_range[0], w.eta_range[1], nt)
    phi = rng.uniform(0.0, 2.0 * np.pi, nt)
    theta = 2.0 * np.arctan(np.exp(-eta))
    tx = np.tan(theta) * np.cos(phi)
    ty = np.tan(theta) * np.sin(phi)
    # track x plane grid
    dz = zp[None, :] - vz[:, None]                       # (nt, P)
    eff = rng.uniform(0.0, 1.0, dz.shape) < w.hit_efficiency
    sx = rng.normal(0.0, w.smear_xy, dz.shape)
    sy = rng.normal(0.0, w.smear_xy, dz.shape)
    hx = vx[:, None] + tx[:, None] * dz + sx
    hy = vy[:, None] + ty[:, None] * dz + sy
    mask = (dz > 0.0) & eff
    if w.acceptance is not None:
        rr = np.hypot(hx, hy)
        mask &= (rr >= w.acceptance[0]) & (rr <= w.acceptance[1])
    ti, pi = np.nonzero(mask)
    x = hx[ti, pi]
    y = hy[ti, pi]
    z = zp[pi]
    part = ti.astype(np.int32)
    plane = pi.astype(np.int32)
    part2 = np.full(len(x), -1, np.int32)
    if w.pair_fraction > 0:
        x, y, z, part, plane, part2 = _add_pairs(w, index, seed_space, x, y, z, part, plane, part2, ti, pi,
                                                 vz, zp, mask)
    n_noise = int(round(w.noise_fraction * len(x)))
    r0, r1 = w.noise_annulus
    nr = np.sqrt(rng.uniform(r0 * r0, r1 * r1, n_noise))
    nphi = rng.uniform(0.0, 2.0 * np.pi, n_noise)
    npl = rng.integers(0, w.n_planes, n_noise).astype(np.int32)
    x = np.concatenate([x, nr * np.cos(nphi)])
    y = np.concatenate([y, nr * np.sin(nphi)])
    z = np.concatenate([z, zp[npl]])
    plane = np.concatenate([plane, npl])
    part = np.concatenate([part, np.full(n_noise, -1, np.int32)])
    part2 = np.concatenate([part2, np.full(n_noise, -1, np.int32)])
    order = rng.permutation(len(x))
    if w.hit_order == "readout":
        order = np.lexsort((np.arctan2(y, x), plane))
    elif w.hit_order != "shuffled":
        raise ValueError(f"unknown hit order {w.hit_order!r}")
    return dict(x=x[order].astype(np.float32), y=y[order].astype(np.float32),
                z=z[order].astype(np.float32), plane=plane[order].astype(np.int32),
                particle=part[order].astype(np.int32), particle2=part2[order].astype(np.int32))


def _add_pairs(w: Workload, index: int, seed_space: Optional[int], x, y, z, part, plane, part2, ti, pi, vz, zp,
               mask):
    """Partners of a fraction of the tracks (conversion pairs): partner j of
    parent t shares t's first s hits (particle2 of those hits = j) and then
    follows t's line turned by a small angle about the last shared hit, with
    its own efficiency and smearing.  Draws from a stream of its own, so the
    rest of the event is the one drawn without pairs."""
    rng = np.random.default_rng(np.random.SeedSequence([w.cid if seed_space is None else seed_space, index, 77]))
    nt, P = mask.shape
    u = rng.uniform(0.0, 1.0, nt)
    s = rng.integers(w.pair_shared[0], w.pair_shared[1] + 1, nt)
    ang = rng.uniform(w.pair_angle[0], w.pair_angle[1], nt)
    psi = rng.uniform(0.0, 2.0 * np.pi, nt)
    eff = rng.uniform(0.0, 1.0, (nt, P)) < w.hit_efficiency
    sx = rng.normal(0.0, w.smear_xy, (nt, P))
    sy = rng.normal(0.0, w.smear_xy, (nt, P))
    counts = np.bincount(ti, minlength=nt)                 # hits of each track (ti ascending, planes ascending)
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    t = np.nonzero((u < w.pair_fraction) & (counts >= s + 2))[0]
    last = starts[t] + s[t] - 1                            # the parent's last shared hit
    end = starts[t] + counts[t] - 1                        # the parent's last hit
    z0 = zp[pi[last]]
    span = np.maximum(zp[pi[end]] - z0, 1e-9)
    tx = (x[end] - x[last]) / span + ang[t] * np.cos(psi[t])
    ty = (y[end] - y[last]) / span + ang[t] * np.sin(psi[t])
    dz = zp[None, :] - z0[:, None]
    later = (dz > 0.0) & (zp[None, :] - vz[t][:, None] > 0.0) & eff[t]
    nx = x[last][:, None] + tx[:, None] * dz + sx[t]
    ny = y[last][:, None] + ty[:, None] * dz + sy[t]
    if w.acceptance is not None:
        rr = np.hypot(nx, ny)
        later &= (rr >= w.acceptance[0]) & (rr <= w.acceptance[1])
    has = later.any(1)
    t, last, s_t, later, nx, ny = t[has], last[has], s[t][has], later[has], nx[has], ny[has]
    ids = nt + np.arange(len(t), dtype=np.int32)
    p2 = part2.copy()
    shared = np.repeat(last - s_t + 1, s_t) + (np.arange(int(s_t.sum())) - np.repeat(np.cumsum(s_t) - s_t, s_t))
    p2[shared] = np.repeat(ids, s_t)
    r, c = np.nonzero(later)
    n_new = len(r)
    return (np.concatenate([x, nx[r, c]]), np.concatenate([y, ny[r, c]]), np.concatenate([z, zp[c]]),
            np.concatenate([part, ids[r]]).astype(np.int32), np.concatenate([plane, c.astype(np.int32)]),
            np.concatenate([p2, np.full(n_new, -1, np.int32)]))


def generate_batch(w: Workload, n_events: Optional[int] = None, first: int = 0,
                   seed_space: Optional[int] = None) -> Dict[str, np.ndarray]:
    """Events ``first .. first+n_events-1`` packed back to back (SoA + hit_off)."""
    n = w.n_events if n_events is None else n_events
    evs = [generate_event(w, first + i, seed_space) for i in range(n)]
    counts = np.array([len(e["x"]) for e in evs], dtype=np.int64)
    hit_off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=hit_off[1:])
    out = {k: (np.concatenate([e[k] for e in evs]) if n else np.zeros(0, evs and evs[0][k].dtype or np.float32))
           for k in ("x", "y", "z", "plane", "particle", "particle2")} if n else \
        dict(x=np.zeros(0, np.float32), y=np.zeros(0, np.float32), z=np.zeros(0, np.float32),
             plane=np.zeros(0, np.int32), particle=np.zeros(0, np.int32), particle2=np.zeros(0, np.int32))
    out["hit_off"] = hit_off
    return out


def event_slice(batch: Dict[str, np.ndarray], i: int) -> Dict[str, np.ndarray]:
    a, b = int(batch["hit_off"][i]), int(batch["hit_off"][i + 1])
    return {k: batch[k][a:b] for k in ("x", "y", "z", "plane", "particle", "particle2") if k in batch}


# ----------------------------------------------------------------------------
# weights
# ----------------------------------------------------------------------------

def layer_shapes(w: Workload) -> Dict[str, List[Tuple[int, int]]]:
    """(fan_in, fan_out) of every Linear layer, grouped by network, in order."""
    H, W, D = w.gnn_hidden, w.emb_hidden, w.emb_dim
    emb = [(3, W)] + [(W, W)] * (w.emb_layers - 1) + [(W, D)]
    shapes = {"emb": emb, "node_enc": [(3, H), (H, H)], "edge_enc": [(2 * H, H), (H, H)]}
    for k in range(w.gnn_steps):
        shapes[f"node{k}"] = [(3 * H, H), (H, H)]
        shapes[f"edge{k}"] = [(3 * H, H), (H, H)]
    shapes["cls"] = [(H, H), (H, 1)]
    return shapes


def xavier_weights(w: Workload, seed: Optional[int] = None) -> Dict[str, List[Tuple[np.ndarray, np.ndarray]]]:
    """Xavier-uniform weights (FP64 draw, rounded once to FP32), zero biases.

    Each Linear layer is (W[fan_in, fan_out], b[fan_out]) with y = x W + b.
    """
    s = w.weight_seed if seed is None else seed
    out: Dict[str, List[Tuple[np.ndarray, np.ndarray]]] = {}
    layer = 0
    for net, shapes in layer_shapes(w).items():
        out[net] = []
        for fi, fo in shapes:
            rng = np.random.default_rng(np.random.SeedSequence([s, layer]))
            a = np.sqrt(6.0 / (fi + fo))
            W = rng.uniform(-a, a, (fi, fo)).astype(np.float32)
            out[net].append((W, np.zeros(fo, np.float32)))
            layer += 1
    return out


def prefilter_shapes(hidden: int = 32) -> List[Tuple[int, int]]:
    return [(6, hidden), (hidden, hidden), (hidden, 1)]


def xavier_prefilter(seed: int = 7, hidden: int = 32) -> List[Tuple[np.ndarray, np.ndarray]]:
    out = []
    for layer, (fi, fo) in enumerate(prefilter_shapes(hidden)):
        rng = np.random.default_rng(np.random.SeedSequence([seed, 1000 + layer]))
        a = np.sqrt(6.0 / (fi + fo))
        out.append((rng.uniform(-a, a, (fi, fo)).astype(np.float32), np.zeros(fo, np.float32)))
    return out


def triplet_shapes(w: Workload) -> List[Tuple[int, int]]:
    """Layers of one triplet classifier: 2H -> H, H -> H, H -> 1."""
    H = w.gnn_hidden
    return [(2 * H, H), (H, H), (H, 1)]


def xavier_triplets(w: Workload, seed: Optional[int] = None) -> Dict[str, List[Tuple[np.ndarray, np.ndarray]]]:
    """Xavier-uniform triplet classifiers (articulations "art", elbows "elb"), zero biases."""
    s = (w.weight_seed if seed is None else seed) + 1
    out: Dict[str, List[Tuple[np.ndarray, np.ndarray]]] = {}
    layer = 0
    for head in ("art", "elb"):
        out[head] = []
        for fi, fo in triplet_shapes(w):
            rng = np.random.default_rng(np.random.SeedSequence([s, 2000 + layer]))
            a = np.sqrt(6.0 / (fi + fo))
            out[head].append((rng.uniform(-a, a, (fi, fo)).astype(np.float32), np.zeros(fo, np.float32)))
            layer += 1
    return out


def load_weights(path: str) -> Dict[str, List[Tuple[np.ndarray, np.ndarray]]]:
    """Weights written by train.save (npz, no pickled objects)."""
    z = np.load(path, allow_pickle=False)
    out: Dict[str, List[Tuple[np.ndarray, np.ndarray]]] = {}
    keys = sorted({k.rsplit(".", 2)[0] for k in z.files})
    for net in keys:
        n = len([k for k in z.files if k.startswith(net + ".") and k.endswith(".W")])
        out[net] = [(z[f"{net}.{i}.W"].astype(np.float32), z[f"{net}.{i}.b"].astype(np.float32)) for i in range(n)]
    return out


TRAINED_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")


def trained_weights(w: Workload) -> Dict[str, List[Tuple[np.ndarray, np.ndarray]]]:
    """The committed trained weight set of a workload's network, trained on the GPU by the library
    (``python -m paper_2508_07423_amd.train --workload <name> --out <file>``)."""
    name = {"c1": "c3", "c3": "c3", "c5": "c3", "c2": "c2", "c4": "c2", "c6": "c6"}[w.name]
    return load_weights(os.path.join(TRAINED_DIR, f"{name}_trained.npz"))


def trained_triplets(w: Workload) -> Dict[str, List[Tuple[np.ndarray, np.ndarray]]]:
    """The committed triplet classifiers ("art", "elb"), trained on the GPU by the library together with the
    network of ``trained_weights(C6)`` (``python -m paper_2508_07423_amd.train --workload c6 --triplets ...``)."""
    if w.gnn_hidden != C6.gnn_hidden:
        raise ValueError("trained triplet classifiers exist for the hidden size of the c6 network only")
    return load_weights(os.path.join(TRAINED_DIR, "c6_triplets.npz"))
