"""The schedule of the two-steps-per-pass kernels (csrc/step2.hpp), checked on
the CPU: which first-step value each second-step population reads, in
which LDS slot of its direction class it is held, which halo a workgroup
recomputes, and (D2Q9 with solids) where halfway bounce-back takes the
node's own first-step value instead, on the host's split into mask-free
chunks and shorter masked ones (D2Q9 rows, D3Q19 column chunks).  The schedule is emulated here in
NumPy with the oracle's collision as the per-node map, and the second
step's pulled populations must equal the oracle's state after two steps
(pulled = pre-collision) exactly.  CPU only: the kernels themselves are
checked bit for bit against one step per pass in test_gpu_step2.py.

Schedule (one workgroup, marching along the last axis a: z in 3D, y in 2D):
for plane k it computes the first step (A) on its tile plus a one-node halo
and keeps each direction i in the slots of its class c = e_ia + 1 (1, 2 and
3 slots; 2, 2, 3 with solids), slot = plane index mod slots(c); the second
step (B) for plane k - 1 reads direction i of node x from A node x - e_i in
plane k - 1 - e_ia, i.e. slot (it - c) mod slots(c).
"""
import numpy as np
import pytest

import lbm_inputs as I
from oracle import ptrt as O


def _classes(e, axis, bb=False):
    c = e[:, axis].astype(int) + 1
    slots = [2 if bb else 1, 2, 3]
    count = [int((c == k).sum()) for k in range(3)]
    index = [int((c[:i] == c[i]).sum()) for i in range(len(c))]
    region = [0, slots[0] * count[0], slots[0] * count[0] + slots[1] * count[1]]
    planes = sum(s * n for s, n in zip(slots, count))
    return c, slots, count, index, region, planes


def _collide(lat, h, tp, lam):
    """Oracle collision of populations h [Q, n] (pre -> post)."""
    tm = 0.5 + lam / (tp - 0.5)
    return O.collide(lat, np.ascontiguousarray(h.T), None, tp, tau_minus=tm).T


def _start(lat, shape, tp, lam, solid=None, seed=3):
    """Oracle lattice at t = 0 and the stored (post-collision) state whose
    pull gives its populations: collide them once at every node."""
    rng = np.random.default_rng(seed)
    rho, u = I.random_fields(rng, shape, umax=0.05)
    if lat == O.D2Q9:
        u = u[:2]
    ora = O.Lattice(lat, shape[2], shape[1], shape[0], tp, lam, solid=solid)
    ora.init_equilibrium(rho, u)
    f = ora.populations()
    Q = f.shape[0]
    stored = _collide(lat, f.reshape(Q, -1), tp, lam).reshape(f.shape)
    ora.step(2)
    return stored, ora.populations()


def _two_step_3d(stored, e, tp, lam, BY, zc):
    """k_step2 schedule on D3Q19: 64 x BY columns, chunks of zc planes."""
    Q, nz, ny, nx = stored.shape
    BX, AX, AY = 64, 66, BY + 2
    AP = AX * AY
    cls, slots, count, index, region, planes = _classes(e, 2)
    out = np.full(stored.shape, np.nan)
    ex, ey, ez = (e[:, a].astype(int) for a in range(3))

    def at(c, i_idx, slot, a):
        v = (region[c] + slot * count[c] + i_idx) * AP + a
        assert np.all((v >= 0) & (v < planes * AP))
        return v

    # A nodes: rows 0..AY-1 at ax = 1..64, then the two halo columns
    ax = np.concatenate([np.tile(np.arange(1, 65), AY), np.zeros(AY, int), np.full(AY, AX - 1)])
    ay = np.concatenate([np.repeat(np.arange(AY), 64), np.arange(AY), np.arange(AY)])
    for bz in range((nz + zc - 1) // zc):
        for by in range((ny + BY - 1) // BY):
            for bx in range(nx // BX):
                x0, y0, zs = bx * BX, by * BY, bz * zc
                ze = min(zs + zc, nz)
                lds = np.full(planes * AP, np.nan)
                for it, k in enumerate(range(zs - 1, ze + 1)):
                    gx, gy, gz = (x0 - 1 + ax) % nx, (y0 - 1 + ay) % ny, k % nz
                    raw = np.stack([stored[i, (gz - ez[i]) % nz, (gy - ey[i]) % ny,
                                           (gx - ex[i]) % nx] for i in range(Q)])
                    post = _collide(O.D3Q19, raw, tp, lam)
                    for i in range(Q):
                        lds[at(cls[i], index[i], it % slots[cls[i]], ay * AX + ax)] = post[i]
                    if k < zs + 1:
                        continue
                    bxl = np.tile(np.arange(64), BY)
                    byl = np.repeat(np.arange(BY), 64)
                    h = np.stack([lds[at(cls[i], index[i], (it - cls[i]) % slots[cls[i]],
                                         (byl + 1 - ey[i]) * AX + (bxl + 1 - ex[i]))]
                                  for i in range(Q)])
                    out[:, (k - 1) % nz, (y0 + byl) % ny, x0 + bxl] = h
    return out


@pytest.mark.parametrize("nx,ny,nz,BY,zc", [
    (64, 8, 5, 4, 2), (128, 4, 3, 4, 8), (64, 10, 3, 4, 8), (64, 13, 2, 4, 1), (64, 8, 6, 8, 3)])
def test_d3q19_schedule(nx, ny, nz, BY, zc):
    e, _, _ = O.lattice(O.D3Q19)
    stored, ref = _start(O.D3Q19, (nz, ny, nx), 0.7, 0.25)
    got = _two_step_3d(stored, e, 0.7, 0.25, BY, zc)
    assert not np.isnan(got).any()
    assert np.abs(got - ref).max() < 1e-14


def _two_step_3d_tasks(stored, e, opp, tp, lam, tasks, solid=None):
    """k_step2_list schedule on D3Q19: one workgroup per task (x0, y0, zs,
    ze, masked): 64 x 4 columns, planes zs ... ze - 1; masked tasks keep two
    slots of the e_z = -1 class and apply bounce-back in both steps."""
    Q, nz, ny, nx = stored.shape
    BY, AX, AY = 4, 66, 6
    AP = AX * AY
    m = solid if solid is not None else np.zeros((nz, ny, nx), np.uint8)
    out = np.full(stored.shape, np.nan)
    ex, ey, ez = (e[:, a].astype(int) for a in range(3))
    ax = np.concatenate([np.tile(np.arange(1, 65), AY), np.zeros(AY, int), np.full(AY, AX - 1)])
    ay = np.concatenate([np.repeat(np.arange(AY), 64), np.arange(AY), np.arange(AY)])
    bxl = np.tile(np.arange(64), BY)
    byl = np.repeat(np.arange(BY), 64)
    for x0, y0, zs, ze, masked in tasks:
        cls, slots, count, index, region, planes = _classes(e, 2, masked)

        def at(c, i_idx, slot, a):
            v = (region[c] + slot * count[c] + i_idx) * AP + a
            assert np.all((v >= 0) & (v < planes * AP))
            return v

        lds = np.full(planes * AP, np.nan)
        for it, k in enumerate(range(zs - 1, ze + 1)):
            gx, gy, gz = (x0 - 1 + ax) % nx, (y0 - 1 + ay) % ny, k % nz
            raw = np.empty((Q, len(ax)))
            for i in range(Q):
                sz, sy, sx = (gz - ez[i]) % nz, (gy - ey[i]) % ny, (gx - ex[i]) % nx
                v = stored[i, sz, sy, sx].copy()
                if masked and i:
                    s_ = m[sz, sy, sx] != 0
                    v[s_] = stored[opp[i], gz, gy, gx][s_]
                raw[i] = v
            post = _collide(O.D3Q19, raw, tp, lam)
            for i in range(Q):
                lds[at(cls[i], index[i], it % slots[cls[i]], ay * AX + ax)] = post[i]
            if k < zs + 1:
                continue
            bz_, by_, bx_ = (k - 1) % nz, (y0 + byl) % ny, x0 + bxl
            h = np.empty((Q, len(bxl)))
            for i in range(Q):
                c = cls[i]
                v = lds[at(c, index[i], (it - c) % slots[c],
                           (byl + 1 - ey[i]) * AX + (bxl + 1 - ex[i]))].copy()
                if masked and i:
                    s_ = m[(bz_ - ez[i]) % nz, (by_ - ey[i]) % ny, (bx_ - ex[i]) % nx] != 0
                    io = opp[i]
                    own = lds[at(cls[io], index[io], (it - 1) % slots[cls[io]],
                                 (byl + 1) * AX + (bxl + 1))]
                    v[s_] = own[s_]
                h[i] = v
            if masked:
                h[:, m[bz_, by_, bx_] != 0] = np.nan
            out[:, bz_, by_, bx_] = h
    return out


def _tasks_3d(shape, zc, zm, solid=None):
    """(x0, y0, zs, ze, masked) as the host builds them: 64 x 4 columns,
    chunks of zc planes; a chunk whose first-step rows y0 - 1 ... y0 + 4,
    zs - 1 ... ze have a solid within one row is masked and split into
    chunks of zm planes."""
    nz, ny, nx = shape
    near = np.zeros((nz, ny), bool)
    if solid is not None:
        sr = solid.any(axis=2)
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                near |= np.roll(np.roll(sr, dz, 0), dy, 1)
    out = []
    for zs in range(0, nz, zc):
        ze = min(zs + zc, nz)
        for y0 in range(0, ny, 4):
            nr = near[np.ix_([z % nz for z in range(zs - 1, ze + 1)],
                             [y % ny for y in range(y0 - 1, y0 + 5)])].any()
            for x0 in range(0, nx, 64):
                if not nr:
                    out.append((x0, y0, zs, ze, False))
                else:
                    out += [(x0, y0, z, min(z + zm, ze), True) for z in range(zs, ze, zm)]
    return out


def _masks_3d():
    rng = np.random.default_rng(5)
    m1 = np.zeros((6, 16, 64), np.uint8)
    m1[:, 0, :] = m1[:, -1, :] = 1
    m2 = np.zeros((7, 10, 64), np.uint8)
    m2[2:4, 3:6, 10:14] = 1
    m2[4, 7, 0] = m2[4, 7, 63] = 1
    m3 = (rng.random((5, 12, 64)) < 0.03).astype(np.uint8)
    # a solid one row outside the first-step rows of the chunk at y0 = 8
    # (rows 7 ... 12) and one plane below the chunk at zs = 4 (planes 3 ... 6)
    m4 = np.zeros((6, 16, 64), np.uint8)
    m4[2, 6, 10:13] = 1
    return [(m1, 3, 2), (m2, 4, 1), (m3, 5, 2), (m4, 2, 1)]


@pytest.mark.parametrize("case", range(4))
@pytest.mark.parametrize("masked_everywhere", [False, True])
def test_d3q19_schedule_solids(case, masked_everywhere):
    """Bounce-back in both steps on the masked column chunks (shorter z
    chunks, the e_z = -1 class with two slots); the mask-free code on the
    others changes nothing (against every chunk masked)."""
    mask, zc, zm = _masks_3d()[case]
    e, _, opp = O.lattice(O.D3Q19)
    tasks = _tasks_3d(mask.shape, zc, zm, np.ones_like(mask) if masked_everywhere else mask)
    assert any(t[4] for t in tasks)
    stored, ref = _start(O.D3Q19, mask.shape, 0.8, 3 / 16, solid=mask)
    got = _two_step_3d_tasks(stored, e, opp, 0.8, 3 / 16, tasks, solid=mask)
    fluid = np.broadcast_to(mask == 0, got.shape)
    assert not np.isnan(got[fluid]).any()
    assert np.abs(got[fluid] - ref[fluid]).max() < 1e-14


def _tasks_2d(ny, nx, yc, near=None, ym=None):
    """(x0, ys, ye, masked) tasks as the host builds them: strips of 62
    columns times chunks of yc rows; with solids, a chunk with a solid
    within one row of its rows ys - 1 ... ye is masked and its rows are
    split into chunks of ym rows (the last partial)."""
    out = []
    for ys in range(0, ny, yc):
        ye = min(ys + yc, ny)
        masked = near is not None and any(near[y % ny] for y in range(ys - 1, ye + 1))
        parts = [(y, min(y + ym, ye)) for y in range(ys, ye, ym)] if masked else [(ys, ye)]
        for a, b in parts:
            for x0 in range(0, nx, 62):
                out.append((x0, a, b, masked))
    return out


def _two_step_2d(stored, e, opp, tp, lam, tasks, solid=None):
    """k_step2_2d schedule on D2Q9: one wave per task (a strip of 62
    columns, 64 A nodes, and rows ys ... ye - 1); masked tasks apply
    bounce-back in both steps."""
    Q, _, ny, nx = stored.shape
    st = stored[:, 0]
    W, BX = 64, 62
    bb = solid is not None
    cls, slots, count, index, region, planes = _classes(e, 1, bb)
    m = solid[0] if bb else np.zeros((ny, nx), bool)
    out = np.full((Q, ny, nx), np.nan)
    lanes = np.arange(W)

    def at(c, i_idx, slot, a):
        v = (region[c] + slot * count[c] + i_idx) * W + a
        assert np.all((v >= 0) & (v < planes * W))
        return v

    for x0, ys, ye, masked in tasks:
        assert not masked or bb
        ax = (x0 - 1 + lanes) % nx
        lds = np.full(planes * W, np.nan)
        for it, k in enumerate(range(ys - 1, ye + 1)):
            raw = np.empty((Q, W))
            for i in range(Q):
                sy, sx = (k - int(e[i, 1])) % ny, (ax - int(e[i, 0])) % nx
                v = st[i, sy, sx].copy()
                if masked and i:
                    s = m[sy, sx] != 0
                    v[s] = st[opp[i], k % ny, ax][s]
                raw[i] = v
            post = _collide(O.D2Q9, raw, tp, lam)
            for i in range(Q):
                lds[at(cls[i], index[i], it % slots[cls[i]], lanes)] = post[i]
            if k < ys + 1:
                continue
            bl = np.arange(1, BX + 1)
            bl = bl[x0 - 1 + bl < nx]
            xb = ax[bl]
            h = np.empty((Q, len(bl)))
            for i in range(Q):
                c = cls[i]
                v = lds[at(c, index[i], (it - c) % slots[c], bl - int(e[i, 0]))].copy()
                if masked and i:
                    s = m[(k - 1 - int(e[i, 1])) % ny, (xb - int(e[i, 0])) % nx] != 0
                    io = opp[i]
                    v[s] = lds[at(cls[io], index[io], (it - 1) % slots[cls[io]], bl)][s]
                h[i] = v
            if masked:
                h[:, m[(k - 1) % ny, xb] != 0] = np.nan
            out[:, (k - 1) % ny, xb] = h
    return out


@pytest.mark.parametrize("ny,nx,yc", [(16, 64, 8), (37, 130, 8), (9, 200, 4), (1, 70, 8),
                                      (2, 5, 8), (33, 17, 3), (30, 1, 8), (1, 1, 1), (5, 1, 1),
                                      (16, 64, 1), (9, 130, 2), (23, 70, 5), (20, 63, 9)])
def test_d2q9_schedule(ny, nx, yc):
    e, _, opp = O.lattice(O.D2Q9)
    stored, ref = _start(O.D2Q9, (1, ny, nx), 0.7, 0.25)
    got = _two_step_2d(stored, e, opp, 0.7, 0.25, _tasks_2d(ny, nx, yc))
    assert not np.isnan(got).any()
    assert np.abs(got - ref[:, 0]).max() < 1e-14


def _masks():
    rng = np.random.default_rng(0)
    m1 = np.zeros((40, 130), np.uint8)
    m1[0] = m1[-1] = 1
    m2 = (rng.random((37, 70)) < 0.08).astype(np.uint8)
    m3 = np.zeros((30, 62), np.uint8)
    m3[10:15, 20:30] = 1
    m3[:, 0] = 1
    m4 = (rng.random((9, 17)) < 0.2).astype(np.uint8)
    m5 = np.zeros((16, 64), np.uint8)
    m5[0] = m5[-1] = 1
    m6 = np.zeros((25, 70), np.uint8)
    m6[10:14] = rng.random((4, 70)) < 0.1
    # (mask, rows per chunk, rows per masked chunk)
    return [(m1, 8, 1), (m2, 8, 3), (m3, 8, 2), (m4, 4, 1), (m5, 1, 1), (m6, 3, 2), (m1, 7, 5)]


def _near_rows(m):
    ny = m.shape[0]
    r = m.any(axis=1)
    return [bool(r[(y - 1) % ny] or r[y] or r[(y + 1) % ny]) for y in range(ny)]


@pytest.mark.parametrize("case", range(7))
@pytest.mark.parametrize("masked_everywhere", [False, True])
def test_d2q9_schedule_solids(case, masked_everywhere):
    """Bounce-back in both steps on the masked tasks, whose rows are split
    into shorter chunks; the mask-free code on chunks with no solid within
    one row changes nothing (against every task masked)."""
    mask, yc, ym = _masks()[case]
    ny, nx = mask.shape
    e, _, opp = O.lattice(O.D2Q9)
    near = [True] * ny if masked_everywhere else _near_rows(mask)
    tasks = _tasks_2d(ny, nx, yc, near, ym)
    assert any(t[3] for t in tasks)
    stored, ref = _start(O.D2Q9, (1, ny, nx), 0.8, 3 / 16, solid=mask[None])
    got = _two_step_2d(stored, e, opp, 0.8, 3 / 16, tasks, solid=mask[None])
    fluid = mask == 0
    assert not np.isnan(got[:, fluid]).any()
    assert np.abs(got[:, fluid] - ref[:, 0][:, fluid]).max() < 1e-14
