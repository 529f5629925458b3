"""Standard 3DGS PLY files <-> stored-form arrays.

A trained 3D Gaussian Splatting scene is a binary little-endian PLY with one
vertex element per splat and float properties, in this order:
x y z, nx ny nz (unused normals), f_dc_0..2, f_rest_0..44, opacity (logit),
scale_0..2 (log standard deviations), rot_0..3 (quaternion w, x, y, z).
The library's stored form (include/nanogs.h, nanogs_gaussians) keeps exactly
these fields, with the 48 SH coefficients in file order (f_dc then f_rest),
so reading and writing are copies.  Extra float properties are ignored on
read; normals are written as zeros.
"""
from __future__ import annotations

import numpy as np

SH_REST = 45
FIELDS = (["x", "y", "z", "nx", "ny", "nz"] + [f"f_dc_{i}" for i in range(3)]
          + [f"f_rest_{i}" for i in range(SH_REST)] + ["opacity"]
          + [f"scale_{i}" for i in range(3)] + [f"rot_{i}" for i in range(4)])
_TYPES = {"float": "f4", "float32": "f4", "double": "f8", "float64": "f8", "uchar": "u1",
          "uint8": "u1", "char": "i1", "int8": "i1", "short": "i2", "int16": "i2",
          "ushort": "u2", "uint16": "u2", "int": "i4", "int32": "i4", "uint": "u4",
          "uint32": "u4"}


def _parse_header(fh):
    line = fh.readline()
    if line.strip() != b"ply":
        raise ValueError("not a PLY file")
    fmt, n, props, in_vertex = None, None, [], False
    while True:
        line = fh.readline()
        if not line:
            raise ValueError("PLY header has no end_header")
        tok = line.decode("ascii", "replace").split()
        if not tok:
            continue
        if tok[0] == "format":
            fmt = tok[1]
        elif tok[0] == "element":
            in_vertex = tok[1] == "vertex"
            if in_vertex:
                n = int(tok[2])
            elif n is None:
                raise ValueError("elements before 'vertex' are not supported")
        elif tok[0] == "property" and in_vertex:
            if tok[1] == "list":
                raise ValueError("list properties in the vertex element are not supported")
            if tok[1] not in _TYPES:
                raise ValueError(f"unknown property type {tok[1]}")
            props.append((tok[2], _TYPES[tok[1]]))
        elif tok[0] == "end_header":
            break
    if fmt != "binary_little_endian":
        raise ValueError(f"only binary_little_endian PLY is supported (got {fmt})")
    if n is None:
        raise ValueError("PLY file has no vertex element")
    return n, props


def read_ply(path: str):
    """Returns (pos[n,3], log_scale[n,3], rot[n,4], opacity[n], sh[n,48]) as
    contiguous float32 arrays."""
    with open(path, "rb") as fh:
        n, props = _parse_header(fh)
        dt = np.dtype([(name, "<" + t) for name, t in props])
        data = np.fromfile(fh, dtype=dt, count=n)
    if data.shape[0] != n:
        raise ValueError(f"PLY file holds {data.shape[0]} of {n} vertices")
    names = set(dt.names)
    need = [f for f in FIELDS if not f.startswith("n")]
    missing = [f for f in need if f not in names]
    if missing:
        raise ValueError(f"PLY file lacks 3DGS properties: {missing[:6]}")

    def cols(keys):
        return np.ascontiguousarray(np.stack([data[k] for k in keys], axis=1).astype(np.float32))

    pos = cols(["x", "y", "z"])
    log_scale = cols([f"scale_{i}" for i in range(3)])
    rot = cols([f"rot_{i}" for i in range(4)])
    opacity = np.ascontiguousarray(data["opacity"].astype(np.float32))
    sh = cols([f"f_dc_{i}" for i in range(3)] + [f"f_rest_{i}" for i in range(SH_REST)])
    return pos, log_scale, rot, opacity, sh


def write_ply(path: str, pos, log_scale, rot, opacity, sh) -> None:
    """Writes stored-form arrays as a standard 3DGS PLY (normals zero)."""
    pos = np.asarray(pos, np.float32)
    n = pos.shape[0]
    cols = {"x": pos[:, 0], "y": pos[:, 1], "z": pos[:, 2]}
    zero = np.zeros(n, np.float32)
    cols.update(nx=zero, ny=zero, nz=zero)
    sh = np.asarray(sh, np.float32).reshape(n, 48)
    for i in range(3):
        cols[f"f_dc_{i}"] = sh[:, i]
    for i in range(SH_REST):
        cols[f"f_rest_{i}"] = sh[:, 3 + i]
    cols["opacity"] = np.asarray(opacity, np.float32).reshape(n)
    ls = np.asarray(log_scale, np.float32).reshape(n, 3)
    r = np.asarray(rot, np.float32).reshape(n, 4)
    for i in range(3):
        cols[f"scale_{i}"] = ls[:, i]
    for i in range(4):
        cols[f"rot_{i}"] = r[:, i]
    dt = np.dtype([(f, "<f4") for f in FIELDS])
    out = np.empty(n, dtype=dt)
    for f in FIELDS:
        out[f] = cols[f]
    header = ["ply", "format binary_little_endian 1.0", f"element vertex {n}"]
    header += [f"property float {f}" for f in FIELDS]
    header += ["end_header"]
    with open(path, "wb") as fh:
        fh.write(("\n".join(header) + "\n").encode("ascii"))
        out.tofile(fh)
