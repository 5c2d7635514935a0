"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the method: only voxel masks (geometry),
material parameters and random current vectors.  Seeds follow
``1000 + workload index``.  The structures stand in for the paper's examples
(thin-film inductors, Sec. III.A; the 90-degree bend, Sec. III.C; a layered
register subsystem, Sec. III.D), whose layouts are not available.

Masks are uint8 arrays indexed [z, y, x] (x fastest in memory).
"""
from __future__ import annotations

import numpy as np

MU0 = 4.0e-7 * np.pi


def rng(seed):
    return np.random.default_rng(seed)


def random_currents(seed, shape, dtype=np.complex128):
    """i.i.d. N(0,1) real and imaginary parts."""
    g = rng(seed)
    x = g.standard_normal(shape) + 1j * g.standard_normal(shape)
    return x.astype(dtype)


def full_box(Kx, Ky, Kz):
    return np.ones((Kz, Ky, Kx), dtype=np.uint8)


def random_mask(seed, Kx, Ky, Kz, fill=0.5):
    """Random voxel occupancy (parity tests of the scatter/gather paths)."""
    g = rng(seed)
    m = (g.random((Kz, Ky, Kx)) < fill).astype(np.uint8)
    if m.sum() == 0:
        m[0, 0, 0] = 1
    return m


def compact_index(mask):
    """Compact voxel numbering of a [Kz, Ky, Kx] mask (x fastest, then y, then
    z): array of the same shape, -1 at empty voxels."""
    idx = np.full(mask.shape, -1, dtype=np.int64)
    nz = mask.reshape(-1) != 0
    idx.reshape(-1)[nz] = np.arange(int(nz.sum()))
    return idx


def _face_list(mask, region, face):
    """(compact voxel index, face code) for the non-empty voxels of the
    [z, y, x] slice `region`."""
    idx = compact_index(mask)[region]
    return [(int(k), face) for k in idx.reshape(-1) if k >= 0]


def _meander(seed, Kx, Ky, Kz, width, thick, gap, z0):
    g = rng(seed)
    m = np.zeros((Kz, Ky, Kx), dtype=np.uint8)
    nl = int(g.integers(5, 8))
    pitch = width + gap
    x0, x1 = 4, Kx - 4
    y0 = (Ky - (nl * pitch - gap)) // 2
    for i in range(nl):
        ys = y0 + i * pitch
        m[z0:z0 + thick, ys:ys + width, x0:x1] = 1
        if i + 1 < nl:
            if i % 2 == 0:
                m[z0:z0 + thick, ys:ys + pitch + width, x1 - width:x1] = 1
            else:
                m[z0:z0 + thick, ys:ys + pitch + width, x0:x0 + width] = 1
    # terminals: the free ends of the first and the last lane
    zs, first = slice(z0, z0 + thick), slice(y0, y0 + width)
    last = slice(y0 + (nl - 1) * pitch, y0 + (nl - 1) * pitch + width)
    plus = _face_list(m, (zs, first, slice(x0, x0 + 1)), 0)
    if (nl - 2) % 2 == 0:   # last lane joined on the right: free end on the left
        minus = _face_list(m, (zs, last, slice(x0, x0 + 1)), 0)
    else:
        minus = _face_list(m, (zs, last, slice(x1 - 1, x1)), 1)
    return m, [(plus, minus)]


def meander(seed, Kx=64, Ky=64, Kz=16, width=4, thick=2, gap=4, z0=7):
    """Meander thin-film inductor: ``n`` horizontal lanes joined alternately at
    the left and right ends (5-7 lanes, seeded)."""
    return _meander(seed, Kx, Ky, Kz, width, thick, gap, z0)[0]


def meander_with_port(seed, Kx=64, Ky=64, Kz=16, width=4, thick=2, gap=4, z0=7):
    """The meander and its one port: + terminal on the outer end face of the
    first lane, - terminal on the free end face of the last lane."""
    return _meander(seed, Kx, Ky, Kz, width, thick, gap, z0)


def _gap_port(m, ys, xs, zvia, zgnd):
    """Port across a one-voxel gap: + on the -z faces of the via voxels at
    z = zvia, - on the +z faces of the ground voxels at z = zgnd below."""
    return (_face_list(m, (slice(zvia, zvia + 1), ys, xs), 4),
            _face_list(m, (slice(zgnd, zgnd + 1), ys, xs), 5))


def ground_with_holes(g, m, z0, z1, nholes, hmin, hmax, keep=()):
    """Ground slab z in [z0, z1) with nholes random rectangular holes; a hole
    that would touch one of the `keep` rectangles (y0, y1, x0, x1) grown by
    one voxel is drawn again."""
    Kz, Ky, Kx = m.shape
    m[z0:z1, :, :] = 1
    made = 0
    while made < nholes:
        hx, hy = int(g.integers(hmin, hmax + 1)), int(g.integers(hmin, hmax + 1))
        x, y = int(g.integers(0, Kx - hx)), int(g.integers(0, Ky - hy))
        if any(y < y1 + 1 and y0 - 1 < y + hy and x < x1 + 1 and x0 - 1 < x + hx for y0, y1, x0, x1 in keep):
            continue
        m[z0:z1, y:y + hy, x:x + hx] = 0
        made += 1


def _connected(m):
    """True if the non-empty voxels form one face-connected piece."""
    idx = np.argwhere(m)
    if idx.size == 0:
        return True
    seen = np.zeros(m.shape, dtype=bool)
    stack = [tuple(idx[0])]
    seen[stack[0]] = True
    count = 0
    while stack:
        z, y, x = stack.pop()
        count += 1
        for dz, dy, dx in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            q = (z + dz, y + dy, x + dx)
            if all(0 <= q[i] < m.shape[i] for i in range(3)) and m[q] and not seen[q]:
                seen[q] = True
                stack.append(q)
    return count == len(idx)


def _strips_over_ground(seed, Kx, Ky, Kz):
    g = rng(seed)
    m = np.zeros((Kz, Ky, Kx), dtype=np.uint8)
    strips = []
    for i in range(16):
        y = 4 + i * (Ky - 8) // 16
        length = int(g.integers(40, 101))
        x = int(g.integers(2, Kx - length - 2))
        strips.append((y, x, length))
    # the holes keep clear of the vias' footprints, so every strip returns
    # through one connected ground
    keep = [r for y, x, n in strips for r in ((y, y + 4, x, x + 4), (y, y + 4, x + n - 4, x + n))]
    ground_with_holes(g, m, 2, 6, 16, 4, 16, keep)
    feet = []
    for y, x, length in strips:
        m[12:14, y:y + 4, x:x + length] = 1
        m[6:12, y:y + 4, x:x + 4] = 1             # shorted via
        m[7:12, y:y + 4, x + length - 4:x + length] = 1  # port via, gap at z=6
        feet.append((slice(y, y + 4), slice(x + length - 4, x + length)))
    assert _connected(m)
    return m, [_gap_port(m, ys, xs, 7, 5) for ys, xs in feet]


def strips_over_ground(seed, Kx=128, Ky=128, Kz=64):
    """Multi-strip inductor over a ground slab with 16 random rectangular holes;
    16 strips (width 4, thickness 2) at z in [12,14), each shorted to ground
    by a via at one end and ending in a via with a one-voxel port gap above
    the ground at the other."""
    return _strips_over_ground(seed, Kx, Ky, Kz)[0]


def strips_over_ground_with_ports(seed, Kx=128, Ky=128, Kz=64):
    """The strips and their 16 ports, one across each via gap (+ on the via's
    bottom faces, - on the ground's top faces below it)."""
    return _strips_over_ground(seed, Kx, Ky, Kz)


def _sharp_bend(seed, Kx, Ky, Kz, width, thick):
    g = rng(seed)
    m = np.zeros((Kz, Ky, Kx), dtype=np.uint8)
    m[2:6, :, :] = 1
    zs = 12
    c = int(g.integers(40, 56))
    m[zs:zs + thick, c:c + width, 8:c + width] = 1
    m[zs:zs + thick, 8:c + width, c:c + width] = 1
    m[6:zs, c:c + width, 8:8 + width] = 1          # shorted via
    m[7:zs, 8:8 + width, c:c + width] = 1          # port via, gap at z=6
    return m, [_gap_port(m, slice(8, 8 + width), slice(c, c + width), 7, 5)]


def sharp_bend(seed, Kx=96, Ky=96, Kz=32, width=6, thick=2):
    """90-degree sharp bend strip over a ground plane (Sec. III.C stand-in)."""
    return _sharp_bend(seed, Kx, Ky, Kz, width, thick)[0]


def sharp_bend_with_port(seed, Kx=96, Ky=96, Kz=32, width=6, thick=2):
    """The bend and its port across the via gap at the end of the y arm."""
    return _sharp_bend(seed, Kx, Ky, Kz, width, thick)


def manhattan_layer(g, m, z0, z1, fill, w=4):
    Kz, Ky, Kx = m.shape
    area = Kx * Ky
    while m[z0].sum() < fill * area:
        length = int(g.integers(16, max(17, Kx // 2)))
        if g.random() < 0.5:
            x = int(g.integers(0, Kx - length)); y = int(g.integers(0, Ky - w))
            m[z0:z1, y:y + w, x:x + length] = 1
        else:
            x = int(g.integers(0, Kx - w)); y = int(g.integers(0, Ky - length))
            m[z0:z1, y:y + length, x:x + w] = 1


def layered_stack(seed, Kx=256, Ky=256, Kz=128):
    """Three-layer stack: ground plane z in [4,12) with 64 holes and two wiring
    layers z in [40,48) and [80,88) of random Manhattan traces at 20 % fill."""
    g = rng(seed)
    m = np.zeros((Kz, Ky, Kx), dtype=np.uint8)
    ground_with_holes(g, m, 4, 12, 64, 4, 16)
    manhattan_layer(g, m, 40, 48, 0.20)
    manhattan_layer(g, m, 80, 88, 0.20)
    return m


def _stack_with_ports(seed, Kx, Ky, Kz):
    g = rng(seed)
    m = np.zeros((Kz, Ky, Kx), dtype=np.uint8)
    strips = []
    for i in range(8):
        y = 8 + i * (Ky - 16) // 8
        length = int(g.integers(60, 121))
        x = int(g.integers(4, Kx - length - 4))
        strips.append((y, x, length))
    keep = [r for y, x, n in strips for r in ((y, y + 4, x, x + 4), (y, y + 4, x + n - 4, x + n))]
    ground_with_holes(g, m, 4, 12, 64, 4, 16, keep)
    manhattan_layer(g, m, 40, 48, 0.20)
    manhattan_layer(g, m, 80, 88, 0.20)
    feet = []
    for y, x, length in strips:
        m[40:48, y:y + 4, x:x + length] = 1          # port trace in the lower wiring layer
        m[12:40, y:y + 4, x:x + 4] = 1               # shorted via down to the ground plane
        m[13:40, y:y + 4, x + length - 4:x + length] = 1  # port via, gap at z = 12
        feet.append((slice(y, y + 4), slice(x + length - 4, x + length)))
    return m, [_gap_port(m, ys, xs, 13, 11) for ys, xs in feet]


def layered_stack_with_ports(seed, Kx=256, Ky=256, Kz=128):
    """The three-layer stack with 8 ports: 8 traces (width 4, length 60-120)
    in the lower wiring layer, each shorted to the ground plane by a via at
    one end and ending in a via with a one-voxel port gap above the ground at
    the other (the ground's holes keep clear of the via footprints).  The
    other traces float; every floating piece is a conductor region of its
    own."""
    return _stack_with_ports(seed, Kx, Ky, Kz)


def strip_array(nstrip=16, length=256, width=4, thick=4, gap=4):
    """Parallel x-directed strips (coupled lines), one port per strip: + terminal
    on the -x end faces, - terminal on the +x end faces.  Returns (mask, ports)
    with ports as lists of (voxel index in compact order, face code) pairs."""
    Ky = nstrip * (width + gap)
    mask = np.zeros((thick, Ky, length), dtype=np.uint8)
    for i in range(nstrip):
        mask[:, i * (width + gap):i * (width + gap) + width, :] = 1
    zz, yy, xx = np.nonzero(mask)
    order = np.lexsort((xx, yy, zz))
    xx, yy = xx[order], yy[order]
    ports = []
    for i in range(nstrip):
        sel = (yy >= i * (width + gap)) & (yy < i * (width + gap) + width)
        plus = [(int(k), 0) for k in np.nonzero(sel & (xx == 0))[0]]
        minus = [(int(k), 1) for k in np.nonzero(sel & (xx == length - 1))[0]]
        ports.append((plus, minus))
    return mask, ports


def square_bend(width, arm):
    """90-degree bend of square cross-section (width voxels) with arms of
    `arm` voxels: one arm along x at y < width, one along y at x >= arm -
    width.  One port: + on the -x end faces of the x arm, - on the +y end
    faces of the y arm.  Returns (mask, ports) like strip_array."""
    mask = np.zeros((width, arm, arm), dtype=np.uint8)
    mask[:, 0:width, :] = 1
    mask[:, :, arm - width:arm] = 1
    zz, yy, xx = np.nonzero(mask)
    order = np.lexsort((xx, yy, zz))
    xx, yy = xx[order], yy[order]
    plus = [(int(k), 0) for k in np.nonzero(xx == 0)[0]]
    minus = [(int(k), 3) for k in np.nonzero(yy == arm - 1)[0]]
    return mask, [(plus, minus)]


# Workload table: grid, voxel size, material (sigma0 S/m, London depth m,
# frequencies Hz), RHS count, and the mask generator.
WORKLOADS = {
    "c1_cube8": dict(K=(8, 8, 8), dx=1e-6, sigma0=1e7, lam=90e-9, freqs=[10e9], nrhs=1,
                     mask=lambda: full_box(8, 8, 8), seed=1000),
    "c2_meander": dict(K=(64, 64, 16), dx=0.25e-6, sigma0=1e7, lam=90e-9, freqs=[10e9], nrhs=1,
                       mask=lambda: meander(1001), seed=1001),
    "c3_strips": dict(K=(128, 128, 64), dx=0.25e-6, sigma0=1e7, lam=90e-9, freqs=[10e9], nrhs=16,
                      mask=lambda: strips_over_ground(1002), seed=1002),
    "c4_bend": dict(K=(96, 96, 32), dx=0.25e-6, sigma0=1e7, lam=90e-9, freqs=[10e9], nrhs=1,
                    mask=lambda: sharp_bend(1003), seed=1003),
    "c5_stack": dict(K=(256, 256, 128), dx=0.5e-6, sigma0=1e7, lam=90e-9,
                     freqs=list(1e9 * 50.0 ** (np.arange(8) / 7.0)), nrhs=8,
                     mask=lambda: layered_stack(1004), seed=1004),
    # dense in z (every plane occupied): exercises the padded z-FFT step
    "cube128": dict(K=(128, 128, 128), dx=1e-6, sigma0=1e7, lam=90e-9, freqs=[10e9], nrhs=8,
                    mask=lambda: full_box(128, 128, 128), seed=1005),
}
