"""Seeded synthetic scenes: geometry, segmentation, cameras and parameters.

Inputs of the method (Sec. 4.2 "Scene Parameterization": a triangle mesh with
per-vertex normals, split into objects with constant material and emission
parameters; Sec. 3.4: several calibrated views).  This module only builds
inputs; it holds none of the method's arithmetic, and both the GPU path and
the CPU oracle consume its arrays.

Parameter layout (length P = 7 S + 3 E, float32, raw physical values):
  segment s:  [7s .. 7s+6]     = kd_r, kd_g, kd_b, ks_r, ks_g, ks_b, alpha
  emitter k:  [7S+3k .. +2]    = e_r, e_g, e_b  (radiance of segment emitter_seg[k])
The optimiser works on theta = p / scale, clamped to [lo, hi].

Workloads (all seeded and synthetic; the paper's scenes and datasets are not
used):
  cornell()   - 36 triangles: 5 wall quads, 2 boxes, 1 ceiling emitter quad;
                8 Lambertian segments; one 64x64 view.
  room()      - one 8x3x6 room with 20 subdivided boxes/cylinders, ~50k
                triangles, 32 segments, 4 ceiling emitters, 4 views 320x240.
  apartment() - 2x3 grid of 5x3x5 rooms with doors, ~160 objects, ~500k
                triangles, 128 segments, 8 emitters, 16 views 640x480.
  office_floor() - 4x6 grid of rooms, ~640 objects, ~2M triangles,
                256 segments, 16 emitters, 30 views 640x480.
  furnace(), area_light_plane(), tiny meshes - closed-form test scenes.
"""
import math

import numpy as np


class MeshBuilder:
    def __init__(self):
        self.v, self.n, self.f, self.s = [], [], [], []
        self.nv = 0

    def add(self, verts, normals, faces, seg):
        verts = np.asarray(verts, np.float64).reshape(-1, 3)
        normals = np.asarray(normals, np.float64).reshape(-1, 3)
        faces = np.asarray(faces, np.int64).reshape(-1, 3)
        self.v.append(verts)
        self.n.append(normals)
        self.f.append(faces + self.nv)
        self.s.append(np.full(faces.shape[0], seg, np.int64))
        self.nv += verts.shape[0]

    def quad(self, center, n, hu, hv, seg, nu=1, nv=1, holes=None):
        """Rectangle center +- hu +- hv facing n, split into nu x nv cells.
        holes: list of (u0,u1,v0,v1) in [-1,1] cell-centre coordinates to skip."""
        c = np.asarray(center, np.float64)
        n = np.asarray(n, np.float64)
        hu = np.asarray(hu, np.float64)
        hv = np.asarray(hv, np.float64)
        if np.dot(np.cross(hu, hv), n) < 0:
            hu, hv = hv, hu
            nu, nv = nv, nu
        su = np.linspace(-1.0, 1.0, nu + 1)
        sv = np.linspace(-1.0, 1.0, nv + 1)
        grid = c[None, None, :] + su[:, None, None] * hu[None, None, :] + sv[None, :, None] * hv[None, None, :]
        verts = grid.reshape(-1, 3)
        idx = np.arange((nu + 1) * (nv + 1)).reshape(nu + 1, nv + 1)
        faces = []
        for i in range(nu):
            for j in range(nv):
                if holes:
                    cu = 0.5 * (su[i] + su[i + 1])
                    cv = 0.5 * (sv[j] + sv[j + 1])
                    if any(h[0] <= cu <= h[1] and h[2] <= cv <= h[3] for h in holes):
                        continue
                a, b, cc, d = idx[i, j], idx[i + 1, j], idx[i + 1, j + 1], idx[i, j + 1]
                faces.append((a, b, cc))
                faces.append((a, cc, d))
        nn = np.tile(n / np.linalg.norm(n), (verts.shape[0], 1))
        self.add(verts, nn, np.asarray(faces, np.int64).reshape(-1, 3), seg)

    def box(self, lo, hi, seg, sub=1):
        lo = np.asarray(lo, np.float64)
        hi = np.asarray(hi, np.float64)
        c = 0.5 * (lo + hi)
        h = 0.5 * (hi - lo)
        ex, ey, ez = np.array([h[0], 0, 0]), np.array([0, h[1], 0]), np.array([0, 0, h[2]])
        for ax, (a, b) in enumerate([(ey, ez), (ex, ez), (ex, ey)]):
            for sgn in (1.0, -1.0):
                n = np.zeros(3)
                n[ax] = sgn
                off = np.zeros(3)
                off[ax] = sgn * h[ax]
                self.quad(c + off, n, a, b, seg, sub, sub)

    def cylinder(self, base, r, height, seg, nr=16, nh=1):
        """Vertical cylinder with smooth side normals and flat caps."""
        base = np.asarray(base, np.float64)
        th = np.linspace(0.0, 2.0 * math.pi, nr + 1)[:-1]
        ys = np.linspace(0.0, height, nh + 1)
        ring = np.stack([np.cos(th), np.zeros_like(th), np.sin(th)], 1)
        verts = (base[None, None, :] + r * ring[None, :, :] +
                 ys[:, None, None] * np.array([0, 1.0, 0])[None, None, :]).reshape(-1, 3)
        normals = np.tile(ring, (nh + 1, 1))
        faces = []
        for i in range(nh):
            for j in range(nr):
                a = i * nr + j
                b = i * nr + (j + 1) % nr
                c = (i + 1) * nr + (j + 1) % nr
                d = (i + 1) * nr + j
                # outward facing: normal = cross(e1, e2) points along ring
                faces.append((a, c, b))
                faces.append((a, d, c))
        self.add(verts, normals, np.asarray(faces), seg)
        for yy, sgn in ((height, 1.0), (0.0, -1.0)):
            ctr = base + np.array([0, yy, 0])
            rim = ctr[None, :] + r * ring
            verts = np.vstack([ctr[None, :], rim])
            fc = []
            for j in range(nr):
                a, b = 1 + j, 1 + (j + 1) % nr
                fc.append((0, b, a) if sgn > 0 else (0, a, b))
            nn = np.tile(np.array([0, sgn, 0.0]), (verts.shape[0], 1))
            self.add(verts, nn, np.asarray(fc), seg)

    def arrays(self):
        v = np.vstack(self.v).astype(np.float32)
        n = np.vstack(self.n)
        n = (n / np.linalg.norm(n, axis=1, keepdims=True)).astype(np.float32)
        f = np.vstack(self.f).astype(np.int32)
        s = np.concatenate(self.s).astype(np.int32)
        return v, n, f, s


def look_at(eye, target, up=(0.0, 1.0, 0.0)):
    """cam_to_world (row-major 4x4, column vectors): camera looks down -z."""
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, np.float64))
    right /= np.linalg.norm(right)
    up2 = np.cross(right, fwd)
    M = np.eye(4)
    M[:3, 0] = right
    M[:3, 1] = up2
    M[:3, 2] = -fwd
    M[:3, 3] = eye
    return M.astype(np.float32)


def _param_vectors(S, E, emitter_seg, rng, kd_range, ks_range, a_range, e_range, lambert_only,
                   e_max):
    P = 7 * S + 3 * E
    p = np.zeros(P, np.float64)
    for s in range(S):
        p[7 * s:7 * s + 3] = rng.uniform(*kd_range, size=3)
        if lambert_only:
            p[7 * s + 3:7 * s + 6] = 0.0
            p[7 * s + 6] = 0.5
        else:
            p[7 * s + 3:7 * s + 6] = rng.uniform(*ks_range, size=3)
            p[7 * s + 6] = rng.uniform(*a_range)
    for k in range(E):
        p[7 * S + 3 * k:7 * S + 3 * k + 3] = rng.uniform(*e_range, size=3)
    scale = np.ones(P)
    scale[7 * S:] = e_max
    lo = np.zeros(P)
    hi = np.ones(P)
    trainable = np.ones(P, np.uint8)
    for s in range(S):
        lo[7 * s + 6] = 1e-3
        if lambert_only:
            trainable[7 * s + 3:7 * s + 7] = 0
    return p.astype(np.float32), scale, lo, hi, trainable


def _finish(name, b, S, emitter_seg, cams, params, scale, lo, hi, trainable, render, normals=True):
    v, n, f, s = b.arrays()
    return dict(name=name, verts=v, normals=n if normals else None, tris=f, tri_seg=s,
                num_segments=S, emitter_seg=np.asarray(emitter_seg, np.int32), cams=cams,
                params=params, scale=scale.astype(np.float32), lo=lo.astype(np.float32),
                hi=hi.astype(np.float32), trainable=trainable, render=render)


def init_theta(scene, mode, seed=0):
    """Initial parameters: mode 'half' (theta = 0.5), 'zero', or 'uniform'
    (theta ~ U(lo, hi), seeded).  Untrainable entries keep their true value."""
    p_true = scene["params"].astype(np.float64)
    scale = scene["scale"].astype(np.float64)
    lo, hi = scene["lo"].astype(np.float64), scene["hi"].astype(np.float64)
    tr = scene["trainable"].astype(bool)
    if mode == "half":
        th = np.full_like(p_true, 0.5)
    elif mode == "zero":
        th = np.zeros_like(p_true)
    elif mode == "uniform":
        th = np.random.default_rng(seed).uniform(0.0, 1.0, size=p_true.size)
    else:
        raise ValueError(mode)
    th = np.clip(th, lo, hi)
    p = np.where(tr, th * scale, p_true)
    return p.astype(np.float32)


def cornell(seed=1):
    """Cornell-box-style scene, 36 triangles (unit room, open front)."""
    rng = np.random.default_rng(seed)
    b = MeshBuilder()
    c = np.array([0.5, 0.5, 0.5])
    X, Y, Z = np.array([0.5, 0, 0]), np.array([0, 0.5, 0]), np.array([0, 0, 0.5])
    b.quad(c - Y, [0, 1, 0], X, Z, 0)        # floor
    b.quad(c + Y, [0, -1, 0], X, Z, 1)       # ceiling
    b.quad(c - Z, [0, 0, 1], X, Y, 2)        # back
    b.quad(c - X, [1, 0, 0], Y, Z, 3)        # left
    b.quad(c + X, [-1, 0, 0], Y, Z, 4)       # right
    # two boxes at seeded, non-overlapping floor positions
    sizes = [(0.3, 0.6, 0.3), (0.3, 0.3, 0.3)]
    placed = []
    for i, (sx, sy, sz) in enumerate(sizes):
        for _ in range(1000):
            x0 = rng.uniform(0.05, 0.95 - sx)
            z0 = rng.uniform(0.05, 0.95 - sz)
            if all(x0 + sx + 0.03 < px or px + psx + 0.03 < x0 or z0 + sz + 0.03 < pz or
                   pz + psz + 0.03 < z0 for (px, pz, psx, psz) in placed):
                break
        placed.append((x0, z0, sx, sz))
        b.box([x0, 0.0, z0], [x0 + sx, sy, z0 + sz], 5 + i)
    b.quad([0.5, 1.0 - 1e-3, 0.5], [0, -1, 0], [0.125, 0, 0], [0, 0, 0.125], 7)   # emitter
    S, E = 8, 1
    emitter_seg = [7]
    params, scale, lo, hi, tr = _param_vectors(S, E, emitter_seg, rng, (0.1, 0.9), None, None,
                                               (5.0, 15.0), True, 15.0)
    cams = dict(cam_to_world=look_at([0.5, 0.5, 1.9], [0.5, 0.5, 0.0])[None],
                fov_y=np.array([math.radians(40.0)], np.float32), width=64, height=64)
    render = dict(spp=4, max_depth=3, rr_depth=-1, target_spp=256, iters=50, lr=1e-2,
                  init="half")
    return _finish("cornell", b, S, emitter_seg, cams, params, scale, lo, hi, tr, render,
                   normals=False)


def _building(name, seed, grid, room, n_objects, target_tris, S, E, n_views, W, H, fov_deg,
              render):
    rng = np.random.default_rng(seed)
    gx, gz = grid
    rw, rh, rd = room
    b = MeshBuilder()
    bx, bz = gx * rw, gz * rd
    n_room_segs = 0

    def room_seg():
        nonlocal n_room_segs
        n_room_segs += 1
        return n_room_segs - 1

    # floor and ceiling: one quad per room, two segments for a single room
    floor_segs, ceil_segs, wall_segs = [], [], []
    nroom_surface = 8 if gx * gz == 1 else min(20, 4 + 2 * gx * gz)
    for i in range(nroom_surface):
        room_seg()
    surf = list(range(nroom_surface))
    k = 0
    for ix in range(gx):
        for iz in range(gz):
            cx, cz = (ix + 0.5) * rw, (iz + 0.5) * rd
            if gx * gz == 1:
                # floor split in two halves (two segments)
                b.quad([cx - rw / 4, 0, cz], [0, 1, 0], [rw / 4, 0, 0], [0, 0, rd / 2], surf[0])
                b.quad([cx + rw / 4, 0, cz], [0, 1, 0], [rw / 4, 0, 0], [0, 0, rd / 2], surf[1])
                b.quad([cx, rh, cz], [0, -1, 0], [rw / 2, 0, 0], [0, 0, rd / 2], surf[2])
            else:
                b.quad([cx, 0, cz], [0, 1, 0], [rw / 2, 0, 0], [0, 0, rd / 2],
                       surf[(2 * k) % nroom_surface])
                b.quad([cx, rh, cz], [0, -1, 0], [rw / 2, 0, 0], [0, 0, rd / 2],
                       surf[(2 * k + 1) % nroom_surface])
            k += 1
    # walls: outer walls, and interior walls with a door opening
    door = dict(w=1.0, h=2.1)

    def wall_x(x, z0, z1, seg, with_door, nrm):
        # wall in plane x = const spanning z0..z1, 0..rh
        zc = 0.5 * (z0 + z1)
        hz = 0.5 * (z1 - z0)
        if not with_door:
            b.quad([x, rh / 2, zc], nrm, [0, rh / 2, 0], [0, 0, hz], seg)
            return
        dz = door["w"] / 2
        # left, right parts and lintel
        b.quad([x, rh / 2, 0.5 * (z0 + zc - dz)], nrm, [0, rh / 2, 0], [0, 0, 0.5 * (zc - dz - z0)], seg)
        b.quad([x, rh / 2, 0.5 * (zc + dz + z1)], nrm, [0, rh / 2, 0], [0, 0, 0.5 * (z1 - zc - dz)], seg)
        b.quad([x, 0.5 * (door["h"] + rh), zc], nrm, [0, 0.5 * (rh - door["h"]), 0], [0, 0, dz], seg)

    def wall_z(z, x0, x1, seg, with_door, nrm):
        xc = 0.5 * (x0 + x1)
        hx = 0.5 * (x1 - x0)
        if not with_door:
            b.quad([xc, rh / 2, z], nrm, [hx, 0, 0], [0, rh / 2, 0], seg)
            return
        dx = door["w"] / 2
        b.quad([0.5 * (x0 + xc - dx), rh / 2, z], nrm, [0.5 * (xc - dx - x0), 0, 0], [0, rh / 2, 0], seg)
        b.quad([0.5 * (xc + dx + x1), rh / 2, z], nrm, [0.5 * (x1 - xc - dx), 0, 0], [0, rh / 2, 0], seg)
        b.quad([xc, 0.5 * (door["h"] + rh), z], nrm, [dx, 0, 0], [0, 0.5 * (rh - door["h"]), 0], seg)

    if gx * gz == 1:
        wall_z(0.0, 0.0, bx / 2, surf[3], False, [0, 0, 1])     # back wall, two segments
        wall_z(0.0, bx / 2, bx, surf[4], False, [0, 0, 1])
        wall_z(bz, 0.0, bx, surf[5], False, [0, 0, -1])
        wall_x(0.0, 0.0, bz, surf[6], False, [1, 0, 0])
        wall_x(bx, 0.0, bz, surf[7], False, [-1, 0, 0])
    else:
        ws = 0
        for iz in range(gz):
            wall_x(0.0, iz * rd, (iz + 1) * rd, surf[ws % nroom_surface], False, [1, 0, 0]); ws += 1
            wall_x(bx, iz * rd, (iz + 1) * rd, surf[ws % nroom_surface], False, [-1, 0, 0]); ws += 1
            for ix in range(1, gx):
                wall_x(ix * rw, iz * rd, (iz + 1) * rd, surf[ws % nroom_surface], True, [1, 0, 0]); ws += 1
        for ix in range(gx):
            wall_z(0.0, ix * rw, (ix + 1) * rw, surf[ws % nroom_surface], False, [0, 0, 1]); ws += 1
            wall_z(bz, ix * rw, (ix + 1) * rw, surf[ws % nroom_surface], False, [0, 0, -1]); ws += 1
            for iz in range(1, gz):
                wall_z(iz * rd, ix * rw, (ix + 1) * rw, surf[ws % nroom_surface], True, [0, 0, 1]); ws += 1
    n_obj_segs = S - E - nroom_surface
    obj_seg0 = nroom_surface
    emit_seg0 = S - E
    # objects: boxes and cylinders on the floor, no overlap (rejection sampling)
    rooms = [(ix, iz) for ix in range(gx) for iz in range(gz)]
    placed = []
    objs = []
    margin = 0.25
    for i in range(n_objects):
        ix, iz = rooms[i % len(rooms)]
        for _ in range(2000):
            kind = "box" if rng.uniform() < 0.55 else "cyl"
            if kind == "box":
                sx, sy, sz = rng.uniform(0.3, 1.5, size=3)
                rad = 0.5 * math.hypot(sx, sz)
            else:
                r = rng.uniform(0.1, 0.5)
                hgt = rng.uniform(0.3, 2.0)
                rad = r
            cx = rng.uniform(ix * rw + margin + rad, (ix + 1) * rw - margin - rad)
            cz = rng.uniform(iz * rd + margin + rad, (iz + 1) * rd - margin - rad)
            if all(math.hypot(cx - px, cz - pz) > rad + pr + 0.1 for px, pz, pr in placed):
                break
        placed.append((cx, cz, rad))
        seg = obj_seg0 + (i % n_obj_segs)
        if kind == "box":
            objs.append(("box", [cx - sx / 2, 0.0, cz - sz / 2], [cx + sx / 2, min(sy, rh - 0.2), cz + sz / 2], seg))
        else:
            objs.append(("cyl", [cx, 0.0, cz], r, min(hgt, rh - 0.2), seg))
    # choose subdivision so the total triangle count is near target_tris
    base_tris = sum(x.shape[0] for x in b.f)
    per_obj = max(12, (target_tris - base_tris - 2 * E) / max(1, n_objects))
    for o in objs:
        if o[0] == "box":
            sub = max(1, int(round(math.sqrt(per_obj / 12.0))))
            b.box(o[1], o[2], o[3], sub)
        else:
            # side 2*nr*nh + caps 2*nr; take nh = nr/2
            nr = max(8, int(round(math.sqrt(per_obj + 1.0) - 1.0)))
            nh = max(1, nr // 2)
            nr = max(8, int(round((per_obj / (nh + 1)) / 2.0)))
            b.cylinder(o[1], o[2], o[3], o[4], nr, nh)
    # emitters: ceiling quads 1e-3*height below the ceiling, facing down
    emitter_seg = []
    emitter_pos = []
    for kk in range(E):
        ix, iz = rooms[kk % len(rooms)]
        j = kk // len(rooms)
        per_room = (E + len(rooms) - 1) // len(rooms)
        fx = (j + 1) / (per_room + 1)
        ex = ix * rw + rw * (0.25 + 0.5 * fx)
        ez = iz * rd + rd * rng.uniform(0.3, 0.7)
        b.quad([ex, rh * (1 - 1e-3), ez], [0, -1, 0], [0.3, 0, 0], [0, 0, 0.3], emit_seg0 + kk)
        emitter_seg.append(emit_seg0 + kk)
        emitter_pos.append((ex, ez))
    params, scale, lo, hi, tr = _param_vectors(S, E, emitter_seg, rng, (0.05, 0.9), (0.0, 0.3),
                                               (0.05, 0.8), (2.0, 20.0), False, 20.0)
    # cameras: eye height 1.6 inside a room, away from objects.  The j-th view
    # of a room with an emitter still unseen looks up towards that emitter from
    # at least 2.6 m away (so every emitter is seen directly); the others look
    # across the room.
    room_emitters = {r: [] for r in range(len(rooms))}
    for kk in range(E):
        room_emitters[kk % len(rooms)].append(emitter_pos[kk])
    c2w = []
    for vi in range(n_views):
        ri = vi % len(rooms)
        ix, iz = rooms[ri]
        j = vi // len(rooms)
        aim = room_emitters[ri][j] if j < len(room_emitters[ri]) else None
        for _ in range(5000):
            ex = rng.uniform(ix * rw + 0.4, (ix + 1) * rw - 0.4)
            ez = rng.uniform(iz * rd + 0.4, (iz + 1) * rd - 0.4)
            far = aim is None or math.hypot(ex - aim[0], ez - aim[1]) >= 2.6
            if far and all(math.hypot(ex - px, ez - pz) > pr + 0.3 for px, pz, pr in placed):
                break
        if aim is not None:
            c2w.append(look_at([ex, 1.6, ez], [aim[0], 2.2, aim[1]]))
            continue
        tx = (ix + 0.5) * rw + rng.uniform(-0.3, 0.3) * rw
        tz = (iz + 0.5) * rd + rng.uniform(-0.3, 0.3) * rd
        if math.hypot(tx - ex, tz - ez) < 1.0:
            tx = 2 * (ix + 0.5) * rw - ex
            tz = 2 * (iz + 0.5) * rd - ez
        c2w.append(look_at([ex, 1.6, ez], [tx, rng.uniform(0.5, 1.2), tz]))
    cams = dict(cam_to_world=np.stack(c2w), fov_y=np.full(n_views, math.radians(fov_deg), np.float32),
                width=W, height=H)
    return _finish(name, b, S, emitter_seg, cams, params, scale, lo, hi, tr, render)


def room(seed=2):
    return _building("room", seed, (1, 1), (8.0, 3.0, 6.0), 20, 50000, 32, 4, 4, 320, 240, 60.0,
                     dict(spp=16, max_depth=5, rr_depth=-1, target_spp=256, iters=200, lr=1e-2,
                          init="uniform"))


def apartment(seed=3):
    return _building("apartment", seed, (2, 3), (5.0, 3.0, 5.0), 160, 500000, 128, 8, 16, 640,
                     480, 60.0,
                     dict(spp=8, max_depth=7, rr_depth=3, target_spp=256, iters=200, lr=1e-2,
                          init="uniform"))


def office_floor(seed=5):
    return _building("office_floor", seed, (4, 6), (5.0, 3.0, 5.0), 640, 2000000, 256, 16, 30,
                     640, 480, 60.0,
                     dict(spp=64, max_depth=8, rr_depth=3, target_spp=128, iters=500, lr=1e-2,
                          init="uniform"))


WORKLOADS = {"cornell": cornell, "room": room, "apartment": apartment,
             "office_floor": office_floor}


def all_emissive(sc):
    """The paper's setting: every segment has an unknown emission (most of it
    zero; the emission of the scene's own emitters keeps its value, the rest
    is 0) besides its material.  Same geometry and cameras; the parameter
    vector grows to 7 S + 3 S and emission is trainable on every segment."""
    S = sc["num_segments"]
    E0 = len(sc["emitter_seg"])
    p_old, sc_old = sc["params"], sc["scale"]
    e_max = float(sc_old[7 * S]) if E0 else 1.0
    e_true = np.zeros((S, 3), np.float32)
    for k, seg in enumerate(sc["emitter_seg"]):
        e_true[int(seg)] = p_old[7 * S + 3 * k:7 * S + 3 * k + 3]
    P = 10 * S
    params = np.concatenate([p_old[:7 * S], e_true.reshape(-1)]).astype(np.float32)
    scale = np.concatenate([sc_old[:7 * S], np.full(3 * S, e_max, np.float32)]).astype(np.float32)
    lo = np.concatenate([sc["lo"][:7 * S], np.zeros(3 * S, np.float32)]).astype(np.float32)
    hi = np.concatenate([sc["hi"][:7 * S], np.ones(3 * S, np.float32)]).astype(np.float32)
    tr = np.concatenate([sc["trainable"][:7 * S], np.ones(3 * S, np.uint8)]).astype(np.uint8)
    out = dict(sc)
    out.update(name=sc["name"] + "_all_emissive", emitter_seg=np.arange(S, dtype=np.int32), params=params,
               scale=scale, lo=lo, hi=hi, trainable=tr, true_emitters=np.asarray(sc["emitter_seg"], np.int32))
    assert params.size == P
    return out


def per_triangle(sc, tris=None, tri_params=None):
    """Per-triangle refinement (App. E, coarse to fine): every triangle in
    `tris` (default: every triangle of a segment that does not emit) becomes a
    segment of its own with its own material, starting from its old
    segment's values (or from tri_params [T, 7] when given).  Emitter segments
    stay whole, so the emission entries keep their order.  The result has
    `parent` (new segment -> old segment) and `seg_of_tri`."""
    S, E = sc["num_segments"], len(sc["emitter_seg"])
    T = sc["tris"].shape[0]
    old = np.asarray(sc["tri_seg"], np.int64)
    emit = set(int(x) for x in sc["emitter_seg"])
    split = np.zeros(T, bool)
    if tris is None:
        split[:] = [int(x) not in emit for x in old]
    else:
        split[np.asarray(tris, np.int64)] = True
        split &= np.array([int(x) not in emit for x in old])
    # old segments that keep at least one triangle stay segments (first), then
    # one new segment per split triangle
    keep = sorted(set(old[~split].tolist()))
    new_of_old = {o: i for i, o in enumerate(keep)}
    seg = np.empty(T, np.int64)
    parent = list(keep)
    for t in range(T):
        if split[t]:
            seg[t] = len(parent)
            parent.append(int(old[t]))
        else:
            seg[t] = new_of_old[int(old[t])]
    S2 = len(parent)
    P2 = 7 * S2 + 3 * E
    pick = lambda a: np.concatenate([np.asarray(a)[7 * np.asarray(parent)[:, None] + np.arange(7)[None, :]].reshape(-1),
                                     np.asarray(a)[7 * S:]])
    params, scale, lo, hi, tr = (pick(sc[k]) for k in ("params", "scale", "lo", "hi", "trainable"))
    if tri_params is not None:
        tp = np.asarray(tri_params, np.float32)
        for t in np.nonzero(split)[0]:
            params[7 * seg[t]:7 * seg[t] + 7] = tp[t]
    emitter_seg = np.array([new_of_old[int(x)] for x in sc["emitter_seg"]], np.int32)
    out = dict(sc)
    out.update(name=sc["name"] + "_per_triangle", tri_seg=seg.astype(np.int32), num_segments=S2,
               emitter_seg=emitter_seg, params=params.astype(np.float32), scale=scale.astype(np.float32),
               lo=lo.astype(np.float32), hi=hi.astype(np.float32), trainable=tr.astype(np.uint8),
               parent=np.asarray(parent, np.int32), seg_of_tri=seg.astype(np.int32))
    assert params.size == P2
    return out


def subdivide(sc, tris):
    """Splits every triangle in `tris` into four at its edge midpoints (the
    supplement's subdivision of textured regions).  A midpoint is shared by
    the split triangles on both sides of an edge; next to an unsplit
    neighbour it lies on that neighbour's edge.  Children keep their
    parent's segment (and so its material), vertex normals are interpolated
    and renormalised.  The result has `parent_tri` (new triangle -> old)."""
    v = np.asarray(sc["verts"], np.float64)
    nrm = None if sc.get("normals") is None else np.asarray(sc["normals"], np.float64)
    f = np.asarray(sc["tris"], np.int64)
    seg = np.asarray(sc["tri_seg"], np.int64)
    split = np.zeros(f.shape[0], bool)
    split[np.asarray(tris, np.int64)] = True
    verts, norms = [v], [nrm] if nrm is not None else None
    mid = {}
    nv = v.shape[0]

    def midpoint(a, b):
        nonlocal nv
        key = (min(a, b), max(a, b))
        if key not in mid:
            verts.append(0.5 * (v[a] + v[b])[None, :])
            if norms is not None:
                m = nrm[a] + nrm[b]
                norms.append((m / max(np.linalg.norm(m), 1e-30))[None, :])
            mid[key] = nv
            nv += 1
        return mid[key]

    out_f, out_s, parent = [], [], []
    for t in range(f.shape[0]):
        a, b, c = (int(x) for x in f[t])
        if not split[t]:
            out_f.append((a, b, c)); out_s.append(seg[t]); parent.append(t)
            continue
        ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
        for tri in ((a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)):
            out_f.append(tri); out_s.append(seg[t]); parent.append(t)
    out = dict(sc)
    out.update(verts=np.vstack(verts).astype(np.float32),
               normals=None if norms is None else np.vstack(norms).astype(np.float32),
               tris=np.asarray(out_f, np.int32), tri_seg=np.asarray(out_s, np.int32),
               parent_tri=np.asarray(parent, np.int64))
    out.pop("tri_params", None)
    return out


def textured_cornell(seed=1, n=12):
    """Cornell box whose walls and floor carry a texture: each is an n x n
    grid of quads, and the albedo varies per triangle (a smooth two-tone
    pattern per wall), so one constant albedo per object cannot match the
    images while one per triangle can.  Returns the per-object scene (the
    parameters hold each object's mean albedo) with `tri_kd` [T, 3], the true
    albedo of every triangle; `per_triangle(sc, tri_params=...)` with it is
    the ground truth."""
    rng = np.random.default_rng(seed)
    b = MeshBuilder()
    c = np.array([0.5, 0.5, 0.5])
    X, Y, Z = np.array([0.5, 0, 0]), np.array([0, 0.5, 0]), np.array([0, 0, 0.5])
    b.quad(c - Y, [0, 1, 0], X, Z, 0, n, n)        # floor
    b.quad(c + Y, [0, -1, 0], X, Z, 1)             # ceiling
    b.quad(c - Z, [0, 0, 1], X, Y, 2, n, n)        # back
    b.quad(c - X, [1, 0, 0], Y, Z, 3, n, n)        # left
    b.quad(c + X, [-1, 0, 0], Y, Z, 4, n, n)       # right
    b.box([0.15, 0.0, 0.2], [0.45, 0.6, 0.5], 5)
    b.box([0.6, 0.0, 0.55], [0.9, 0.3, 0.85], 6)
    b.quad([0.5, 1.0 - 1e-3, 0.5], [0, -1, 0], [0.125, 0, 0], [0, 0, 0.125], 7)
    S, E = 8, 1
    params, scale, lo, hi, tr = _param_vectors(S, E, [7], rng, (0.2, 0.8), None, None, (5.0, 15.0), True, 15.0)
    v, nrm, f, sg = b.arrays()
    T = f.shape[0]
    # the texture of each textured object: two tones mixed by a seeded sinusoid of position
    tex = {}
    for s_ in (0, 2, 3, 4):
        a, b2 = rng.uniform(0.15, 0.45, 3), rng.uniform(0.55, 0.9, 3)
        k = rng.uniform(4.0, 9.0, 3)
        ph = rng.uniform(0, 2 * math.pi)
        tex[s_] = (a, b2, k, ph)

    def albedo_at(s_, x):
        """True albedo of object s_ at points x [n, 3] (its constant albedo if untextured)."""
        x = np.asarray(x, np.float64).reshape(-1, 3)
        if s_ not in tex:
            return np.repeat(params[7 * s_:7 * s_ + 3][None, :].astype(np.float64), x.shape[0], axis=0)
        a, b2, k, ph = tex[s_]
        w = 0.5 + 0.5 * np.sin(k[0] * x[:, 0] + k[1] * x[:, 1] + k[2] * x[:, 2] + ph)
        return a[None, :] + (b2 - a)[None, :] * w[:, None]

    cen = v[f].mean(axis=1).astype(np.float64)
    tri_kd = np.zeros((T, 3))
    for s_ in range(S):
        m = sg == s_
        if m.any():
            tri_kd[m] = albedo_at(s_, cen[m])
            if s_ in tex:
                params[7 * s_:7 * s_ + 3] = tri_kd[m].mean(axis=0)
    cams = dict(cam_to_world=look_at([0.5, 0.5, 1.9], [0.5, 0.5, 0.0])[None],
                fov_y=np.array([math.radians(40.0)], np.float32), width=128, height=128)
    render = dict(spp=16, max_depth=3, rr_depth=-1, target_spp=1024, iters=300, lr=1e-2, init="half")
    out = dict(name="textured_cornell", verts=v, normals=None, tris=f, tri_seg=sg, num_segments=S,
               emitter_seg=np.array([7], np.int32), cams=cams, params=params,
               scale=scale.astype(np.float32), lo=lo.astype(np.float32), hi=hi.astype(np.float32),
               trainable=tr, render=render)
    tp = np.zeros((T, 7), np.float32)
    tp[:, :3] = tri_kd
    tp[:, 6] = 0.5
    out["tri_params"] = tp
    out["albedo_at"] = albedo_at
    return out


# --------------------------------------------------------------------------
# Closed-form test scenes and tiny meshes.
# --------------------------------------------------------------------------
def furnace(rho=0.5, E=1.0, half=1.0):
    """Closed cube, every face one Lambertian emitting segment (inward facing).
    Camera at the centre."""
    b = MeshBuilder()
    c = np.zeros(3)
    for ax in range(3):
        for sgn in (1.0, -1.0):
            n = np.zeros(3)
            n[ax] = -sgn
            off = np.zeros(3)
            off[ax] = sgn * half
            a, bb = [np.eye(3)[i] * half for i in range(3) if i != ax]
            b.quad(c + off, n, a, bb, 0)
    S, Ecount = 1, 1
    p = np.array([rho, rho, rho, 0, 0, 0, 0.5, E, E, E], np.float32)
    cams = dict(cam_to_world=look_at([0.0, 0.0, 0.0], [0.0, 0.0, -1.0])[None],
                fov_y=np.array([math.radians(60.0)], np.float32), width=8, height=8)
    P = 10
    return dict(name="furnace", verts=b.arrays()[0], normals=None, tris=b.arrays()[2],
                tri_seg=b.arrays()[3], num_segments=S, emitter_seg=np.array([0], np.int32),
                cams=cams, params=p, scale=np.ones(P, np.float32), lo=np.zeros(P, np.float32),
                hi=np.ones(P, np.float32), trainable=np.ones(P, np.uint8), render={})


def area_light_plane(rho=0.6, Le=5.0, light_half=0.5, light_height=1.0, plane_half=20.0):
    """A large Lambertian plane (y = 0, facing up) under a square emitter quad
    (facing down).  Segment 0: plane, segment 1: emitter (kd = 0).
    Camera looks straight down from above the light's side."""
    b = MeshBuilder()
    b.quad([0, 0, 0], [0, 1, 0], [plane_half, 0, 0], [0, 0, plane_half], 0)
    b.quad([0, light_height, 0], [0, -1, 0], [light_half, 0, 0], [0, 0, light_half], 1)
    p = np.array([rho, rho, rho, 0, 0, 0, 0.5, 0, 0, 0, 0, 0, 0, 0.5, Le, Le, Le], np.float32)
    cams = dict(cam_to_world=look_at([2.5, 3.0, 0.3], [1.5, 0.0, 0.2], up=(0, 0, -1))[None],
                fov_y=np.array([math.radians(30.0)], np.float32), width=8, height=8)
    v, n, f, s = b.arrays()
    P = 17
    return dict(name="area_light_plane", verts=v, normals=None, tris=f, tri_seg=s,
                num_segments=2, emitter_seg=np.array([1], np.int32), cams=cams, params=p,
                scale=np.ones(P, np.float32), lo=np.zeros(P, np.float32),
                hi=np.ones(P, np.float32), trainable=np.ones(P, np.uint8), render={})


def random_soup(n, seed=0, extent=1.0):
    """n random triangles in a cube (for hit tests)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-extent, extent, size=(n, 1, 3))
    v = (c + rng.normal(scale=0.15 * extent, size=(n, 3, 3))).reshape(-1, 3).astype(np.float32)
    f = np.arange(3 * n, dtype=np.int32).reshape(n, 3)
    return v, f


# Disney material model (Sec. 4.1: base colour and ten parameters, all in
# [0, 1]): per segment, in this order
DISNEY_PARAMS = ("base_r", "base_g", "base_b", "subsurface", "metallic", "specular", "specular_tint",
                 "roughness", "anisotropic", "sheen", "sheen_tint", "clearcoat", "clearcoat_gloss")


def disney(scene, seed=0):
    """The scene with the Disney material model: 13 parameters per segment
    instead of 7, emission unchanged.  The base colour is the segment's
    diffuse albedo; the other ten are seeded draws: subsurface, specular,
    specular tint, sheen and sheen tint ~ U(0, 1); metallic 0 with
    probability 0.6, else U(0.2, 1); roughness ~ U(0.25, 0.9); anisotropic
    ~ U(0, 0.8); clearcoat 0 with probability 0.5, else U(0, 1); clearcoat
    gloss ~ U(0, 0.7).  Every parameter is trainable with scale 1 and
    bounds [0, 1]; the emission entries keep their scale and bounds."""
    rng = np.random.default_rng(seed)
    S = scene["num_segments"]
    E = len(scene["emitter_seg"])
    p7 = scene["params"][:7 * S].reshape(S, 7).astype(np.float64)
    d = np.zeros((S, 13))
    d[:, 0:3] = p7[:, 0:3]
    d[:, 3] = rng.uniform(0, 1, S)
    d[:, 4] = np.where(rng.random(S) < 0.6, 0.0, rng.uniform(0.2, 1.0, S))
    d[:, 5] = rng.uniform(0, 1, S)
    d[:, 6] = rng.uniform(0, 1, S)
    d[:, 7] = rng.uniform(0.25, 0.9, S)
    d[:, 8] = rng.uniform(0, 0.8, S)
    d[:, 9] = rng.uniform(0, 1, S)
    d[:, 10] = rng.uniform(0, 1, S)
    d[:, 11] = np.where(rng.random(S) < 0.5, 0.0, rng.uniform(0, 1, S))
    d[:, 12] = rng.uniform(0, 0.7, S)
    out = dict(scene)
    out["name"] = scene["name"] + "_disney"
    out["material"] = 1
    out["params"] = np.concatenate([d.reshape(-1), scene["params"][7 * S:]]).astype(np.float32)
    n = 13 * S
    out["scale"] = np.concatenate([np.ones(n), scene["scale"][7 * S:]]).astype(np.float32)
    out["lo"] = np.concatenate([np.zeros(n), scene["lo"][7 * S:]]).astype(np.float32)
    out["hi"] = np.concatenate([np.ones(n), scene["hi"][7 * S:]]).astype(np.float32)
    out["trainable"] = np.concatenate([np.ones(n), scene["trainable"][7 * S:]]).astype(np.uint8)
    assert out["params"].size == 13 * S + 3 * E
    return out


def scene_arrays(scene):
    """The subset of keys ipt_scene_build and the oracle take."""
    return dict(verts=scene["verts"], normals=scene["normals"], tris=scene["tris"],
                tri_seg=scene["tri_seg"], num_segments=scene["num_segments"],
                emitter_seg=scene["emitter_seg"])
