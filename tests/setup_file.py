"""Reader and writer of the setup-file layout that include/ddlr.h documents
for ddlr_export_setup / ddlr_import_setup, written from that description
(no test functions here).  The tests use the writer to hand the oracle's
complete setup to the library and the reader to inspect the library's
export."""
import struct

import numpy as np

MAGIC = b"DDLRSET1"
_TYPES = {1: np.int32, 2: np.int64, 3: np.float64}
_CODES = {np.dtype(np.int32): 1, np.dtype(np.int64): 2, np.dtype(np.float64): 3}


def write(path, records):
    """records: {name: 1-D numpy array of int32 / int64 / float64}."""
    with open(path, "wb") as f:
        f.write(MAGIC)
        f.write(struct.pack("<ii", 1, len(records)))
        for name, arr in records.items():
            a = np.ascontiguousarray(arr)
            code = _CODES[a.dtype]
            raw = name.encode("ascii")
            assert len(raw) <= 15
            f.write(raw + b"\0" * (16 - len(raw)))
            f.write(struct.pack("<iiq", code, 0, a.size))
            f.write(a.astype(a.dtype.newbyteorder("<"), copy=False).tobytes())


def read(path):
    with open(path, "rb") as f:
        data = f.read()
    assert data[:8] == MAGIC, "bad magic"
    version, count = struct.unpack_from("<ii", data, 8)
    assert version == 1
    off, out = 16, {}
    for _ in range(count):
        name = data[off:off + 16].split(b"\0")[0].decode("ascii")
        code, zero, n = struct.unpack_from("<iiq", data, off + 16)
        off += 32
        dt = np.dtype(_TYPES[code]).newbyteorder("<")
        out[name] = np.frombuffer(data, dtype=dt, count=n, offset=off).copy()
        off += n * dt.itemsize
    assert off == len(data), "trailing bytes"
    return out


def from_oracle(o, alpha=1.0, csolve=0, precision=0, cheb_nu=0):
    """The oracle's complete setup in the file layout: ordering, factors,
    levels left out (the library recomputes them), X or the Chebyshev interval,
    and the low-rank part if the oracle has one."""
    perm, iface, colour, boff = o.ordering()
    L = o.csr("L").tocsr()
    D = o.diag().copy()
    rp, ci, v = L.indptr.astype(np.int64), L.indices.astype(np.int32), L.data.astype(np.float64)
    if csolve == 1:  # C_alpha by X: the interface block has no factor
        m = int(boff[-2])
        keep = np.arange(len(ci)) < rp[m]
        ci, v = ci[keep], v[keep]
        rp = np.minimum(rp, rp[m])
        D[m:] = 1.0
    rec = {
        "n_p": np.array([o.n, o.p], np.int64),
        "alpha": np.array([alpha], np.float64),
        "csolve_prec_nu": np.array([csolve, precision, cheb_nu], np.int32),
        "perm": perm.astype(np.int32),
        "boff": boff.astype(np.int64),
        "colour": colour.astype(np.int32),
        "L.rowptr": rp, "L.col": ci, "L.val": v,
        "D": D,
    }
    if csolve == 1:
        X, res, spd = o.cinv()
        rec["X.rowptr"] = X.indptr.astype(np.int64)
        rec["X.col"] = X.indices.astype(np.int32)
        rec["X.val"] = X.data.astype(np.float64)
        rec["X.cert"] = np.array([o.cinv_rinf, 1.0 if spd else 0.0])
        rec["X.res"] = np.asarray(res, np.float64)
    if csolve == 2:
        rec["cheb"] = np.array(o.cheb(), np.float64)
    if o.variant:
        lr = o.get_lowrank()
        U = lr[0]
        aux = np.concatenate([lr[1], [lr[2]]]) if o.variant == 1 else np.asfortranarray(lr[1]).reshape(-1, order="F")
        rec["lowrank"] = np.array([o.variant, o.k], np.int32)
        rec["U"] = np.asfortranarray(U).reshape(-1, order="F").astype(np.float64)
        rec["aux"] = aux.astype(np.float64)
    return rec
