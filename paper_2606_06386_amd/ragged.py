"""Packing of ragged (mixed-precision) division batches for mp_divrem_ragged.

Operands of every instance are laid end to end in one u pool and one v pool
(each instance 4-limb aligned); the quotient and remainder pools are laid out
the same way.  A descriptor per instance (mp_desc_t in include/mpdiv.h) holds
the limb offsets and widths.
"""
import numpy as np

DESC_DTYPE = np.dtype([("u_off", "<i8"), ("v_off", "<i8"), ("q_off", "<i8"), ("r_off", "<i8"),
                       ("nu", "<i4"), ("nv", "<i4"), ("nq", "<i4"), ("reserved", "<i4")])
assert DESC_DTYPE.itemsize == 48


def _offsets(widths):
    w = (np.asarray(widths, dtype=np.int64) + 3) & ~3
    off = np.zeros(len(w) + 1, dtype=np.int64)
    np.cumsum(w, out=off[1:])
    return off


def pack(us, vs, nqs=None):
    """Pools and descriptors for instances (us[j], vs[j]); nq defaults to nu.

    Returns dict(u_pool, v_pool, desc, q_limbs, r_limbs) with numpy arrays."""
    nus = np.array([len(u) for u in us], dtype=np.int64)
    nvs = np.array([len(v) for v in vs], dtype=np.int64)
    nqs = nus.copy() if nqs is None else np.asarray(nqs, dtype=np.int64)
    uo, vo, qo, ro = _offsets(nus), _offsets(nvs), _offsets(nqs), _offsets(nvs)
    u_pool = np.zeros(max(int(uo[-1]), 1), dtype=np.uint32)
    v_pool = np.zeros(max(int(vo[-1]), 1), dtype=np.uint32)
    for j, (u, v) in enumerate(zip(us, vs)):
        u_pool[uo[j]:uo[j] + nus[j]] = u
        v_pool[vo[j]:vo[j] + nvs[j]] = v
    desc = np.zeros(len(us), dtype=DESC_DTYPE)
    desc["u_off"], desc["v_off"], desc["q_off"], desc["r_off"] = uo[:-1], vo[:-1], qo[:-1], ro[:-1]
    desc["nu"], desc["nv"], desc["nq"] = nus, nvs, nqs
    return {"u_pool": u_pool, "v_pool": v_pool, "desc": desc, "q_limbs": max(int(qo[-1]), 1),
            "r_limbs": max(int(ro[-1]), 1)}


def unpack(pool, desc, which):
    """Rows of instance results from a q or r pool ('q' or 'r')."""
    off = desc["q_off"] if which == "q" else desc["r_off"]
    n = desc["nq"] if which == "q" else desc["nv"]
    return [pool[o:o + k] for o, k in zip(off.tolist(), n.tolist())]
