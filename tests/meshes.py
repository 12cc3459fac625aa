"""Tiny hand-built polyhedral meshes for the CPU pins (not generators of the method)."""
import numpy as np


def single_tet(P):
    """One tetrahedron with vertices P (4, 3); every face is a boundary face oriented outward."""
    P = np.asarray(P, dtype=np.float64)
    faces = [[1, 2, 3], [0, 3, 2], [0, 1, 3], [0, 2, 1]]
    # orient each loop so that its normal points away from the opposite vertex
    loops = []
    for opp, f in zip(range(4), faces):
        a, b, c = P[f]
        n = np.cross(b - a, c - a)
        if np.dot(n, a - P[opp]) < 0:
            f = f[::-1]
        loops.append(f)
    return {
        "xyz": P,
        "face_ptr": np.arange(0, 13, 3, dtype=np.int32),
        "face_vtx": np.array(loops, dtype=np.int32).ravel(),
        "cell_ptr": np.array([0, 4], dtype=np.int32),
        "cell_face": np.arange(4, dtype=np.int32),
        "cell_face_sign": np.ones(4, dtype=np.int8),
    }


def single_prism(h=0.7):
    """Right triangular prism: triangle (0,0),(1,0),(0,1) extruded to height h."""
    P = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, h], [1, 0, h], [0, 1, h]], dtype=np.float64)
    loops = [[0, 2, 1], [3, 4, 5], [0, 1, 4, 3], [1, 2, 5, 4], [2, 0, 3, 5]]
    ptr = np.cumsum([0] + [len(l) for l in loops]).astype(np.int32)
    return {
        "xyz": P,
        "face_ptr": ptr,
        "face_vtx": np.concatenate(loops).astype(np.int32),
        "cell_ptr": np.array([0, 5], dtype=np.int32),
        "cell_face": np.arange(5, dtype=np.int32),
        "cell_face_sign": np.ones(5, dtype=np.int8),
    }
