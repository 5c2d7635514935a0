"""Seeded port geometries of the full-size solve workloads (CPU only).

Each structure must be one face-connected conductor (otherwise a port can be
an open circuit and the admittance matrix singular), and every terminal face
must be a free surface: the voxel across it is empty (a via gap or a lane
end), so the + and - terminals are distinct nodes.
"""
import numpy as np
import pytest

import workloads as wl

# face code -> (axis index in [z, y, x] order, step)
_STEP = {0: (2, -1), 1: (2, 1), 2: (1, -1), 3: (1, 1), 4: (0, -1), 5: (0, 1)}

CASES = {
    "meander": lambda: wl.meander_with_port(1001),
    "strips_over_ground": lambda: wl.strips_over_ground_with_ports(1002),
    "bend": lambda: wl.sharp_bend_with_port(1003),
}


def _components(m):
    """Number of face-connected pieces of the non-empty voxels."""
    lab = np.zeros(m.shape, dtype=np.int64)
    n = 0
    for start in map(tuple, np.argwhere(m)):
        if lab[start]:
            continue
        n += 1
        lab[start] = n
        stack = [start]
        while stack:
            p = stack.pop()
            for a, s in _STEP.values():
                q = list(p)
                q[a] += s
                q = tuple(q)
                if 0 <= q[a] < m.shape[a] and m[q] and not lab[q]:
                    lab[q] = n
                    stack.append(q)
    return n


@pytest.mark.parametrize("name", sorted(CASES))
def test_port_geometry(name):
    m, ports = CASES[name]()
    assert _components(m) == 1
    P = np.argwhere(m)  # [z, y, x] in compact order (x fastest)
    assert np.array_equal(wl.compact_index(m)[tuple(P.T)], np.arange(P.shape[0]))
    for plus, minus in ports:
        assert plus and minus
        faces = set()
        for k, f in plus + minus:
            a, s = _STEP[f]
            q = P[k].copy()
            q[a] += s
            assert not (0 <= q[a] < m.shape[a]) or not m[tuple(q)], (name, k, f)
            key = tuple(P[k]) + (f,)
            assert key not in faces
            faces.add(key)


def test_stack_mask_unchanged_by_hole_rule():
    """The hole generator only redraws holes when footprints are given; the
    stack (no footprints) keeps its seeded layout: K = 687,600 voxels on 24
    occupied planes."""
    m = wl.WORKLOADS["c5_stack"]["mask"]()
    assert int(m.sum()) == 687600
    assert int(m.reshape(m.shape[0], -1).any(axis=1).sum()) == 24
