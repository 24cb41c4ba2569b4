"""Mesh skeleton for the oracle (section 2.1: faces E_h = E_h^I U E_h^B).

Conventions (fixed by this implementation and followed by the HIP library's own code):
  * local face f of a simplex is the face opposite its local vertex f;
  * a global face is identified by its sorted global vertex ids (g0 < g1 [< g2]);
    global faces are numbered in lexicographic order of that sorted tuple;
  * each face is parametrised from the reference face (segment [0,1] or triangle
    (0,0),(1,0),(0,1)) by y(s,t) = X_g0 + (X_g1 - X_g0) s + (X_g2 - X_g0) t, so both
    neighbours see the same trace basis on it;
  * interior faces are shared by two elements, boundary faces by one.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Skeleton:
    dim: int
    faces: np.ndarray          # [n_faces, dim] sorted global vertex ids
    elem_faces: np.ndarray     # [n_elem, dim+1] global face id of local face f
    face_elems: np.ndarray     # [n_faces, 2] adjacent elements (-1 if none)
    is_boundary: np.ndarray    # [n_faces] bool

    @property
    def n_faces(self):
        return self.faces.shape[0]


def build_skeleton(elem_vert: np.ndarray) -> Skeleton:
    ne, nv = elem_vert.shape
    dim = nv - 1
    keys = {}
    for e in range(ne):
        for f in range(nv):
            key = tuple(sorted(int(elem_vert[e, v]) for v in range(nv) if v != f))
            keys.setdefault(key, []).append((e, f))
    sorted_keys = sorted(keys)
    index = {key: i for i, key in enumerate(sorted_keys)}
    faces = np.asarray(sorted_keys, dtype=np.int64)
    elem_faces = np.empty((ne, nv), dtype=np.int64)
    face_elems = -np.ones((len(sorted_keys), 2), dtype=np.int64)
    for key, lst in keys.items():
        if len(lst) > 2:
            raise ValueError("non-manifold face")
        i = index[key]
        for slot, (e, f) in enumerate(lst):
            elem_faces[e, f] = i
            face_elems[i, slot] = e
    is_b = face_elems[:, 1] < 0
    return Skeleton(dim, faces, elem_faces, face_elems, is_b)


def element_map(xyz, elem_vert, e):
    """Affine map x = X0 + J xi of element e; returns (X0, J, detJ, Jinv)."""
    X = xyz[elem_vert[e]]
    J = (X[1:] - X[0]).T
    det = np.linalg.det(J)
    return X[0], J, det, np.linalg.inv(J)


def face_map(xyz, face_verts):
    """Canonical face parametrisation: origin and tangent columns (dim x (dim-1))."""
    P = xyz[face_verts]
    return P[0], (P[1:] - P[0]).T


def face_measure_and_normal(xyz, face_verts, elem_centroid):
    """Face measure (length/area) and the unit normal pointing away from elem_centroid."""
    P0, T = face_map(xyz, face_verts)
    dim = P0.shape[0]
    if dim == 2:
        t = T[:, 0]
        nrm = np.array([t[1], -t[0]])
        meas = np.linalg.norm(t)
    else:
        nrm = np.cross(T[:, 0], T[:, 1])
        meas = 0.5 * np.linalg.norm(nrm)
    nrm = nrm / np.linalg.norm(nrm)
    centroid = xyz[face_verts].mean(axis=0)
    if np.dot(nrm, centroid - elem_centroid) < 0:
        nrm = -nrm
    return meas, nrm


def face_frame(xyz, face_verts):
    """Face-owned orthonormal tangent frame (t1, t2) for 3D tangential traces:
    t1 along X_g1 - X_g0, t2 = n_F x t1 with n_F the normal of the canonical
    parametrisation (independent of which element looks at the face)."""
    P0, T = face_map(xyz, face_verts)
    t1 = T[:, 0] / np.linalg.norm(T[:, 0])
    nF = np.cross(T[:, 0], T[:, 1])
    nF = nF / np.linalg.norm(nF)
    t2 = np.cross(nF, t1)
    return t1, t2
