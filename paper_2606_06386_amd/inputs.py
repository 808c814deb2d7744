"""Seeded synthetic inputs for batched multi-precision division.

This module only draws random limbs; it holds none of the division method's
arithmetic.  Both the GPU path's tests/benchmark and the oracle's tests take
their inputs from here, so any instance can be regenerated alone from
(config seed, instance index).

Random source: splitmix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), used in its counter form: output i of a
generator started at state s is mix(s + (i + 1) * GAMMA).  A 32-bit limb is
the high half of one output.

Instance j of a configuration seeded with ``seed`` has base state
``seed XOR (j * GAMMA mod 2^64)``; it draws from independent sub-streams
(the base generator's outputs 0, 1, 2, ... are the sub-stream states):
  stream 0: limbs of u,  stream 1: limbs of v,  stream 2: per-instance
  sizes and choices,  stream 3: extra operands (the w of u = v*w + v - 1).
"Top limb nonzero" means: if the top limb drawn is 0, it is replaced by the
first nonzero draw after the operand's own draws in the same stream.

Workloads follow the paper's evaluation (random integers, Sec. 4, "Datasets"
and "Methodology") at the precisions 2^15 .. 2^18 bits with 32-bit limbs.
"""
import numpy as np

GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1

SEED_BASE = 0xD1500000

# named workloads: seed = SEED_BASE + index
SEED_C1, SEED_C2, SEED_C3, SEED_C4, SEED_C5 = (SEED_BASE + i for i in range(1, 6))


def _mix(z):
    """splitmix64 output function on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
    return z ^ (z >> np.uint64(31))


def draws(states, start, count):
    """Outputs start .. start+count-1 of each generator in ``states`` -> [len, count] uint64."""
    states = np.asarray(states, dtype=np.uint64).reshape(-1)
    idx = (np.arange(start + 1, start + count + 1, dtype=np.uint64))
    with np.errstate(over="ignore"):
        z = states[:, None] + idx[None, :] * np.uint64(GAMMA)
    return _mix(z)


def instance_states(seed, index):
    """Base generator state of instance(s) ``index`` of a config seeded ``seed``."""
    index = np.asarray(index, dtype=np.uint64).reshape(-1)
    with np.errstate(over="ignore"):
        return np.uint64(seed & MASK64) ^ (index * np.uint64(GAMMA))


def substream(states, t):
    """State of sub-stream t of each base generator."""
    return draws(states, t, 1)[:, 0]


def limbs(states, n):
    """n uniform 32-bit limbs per generator -> [len, n] uint32."""
    if n == 0:
        return np.zeros((len(np.atleast_1d(states)), 0), dtype=np.uint32)
    return (draws(states, 0, n) >> np.uint64(32)).astype(np.uint32)


def limbs_top_nonzero(states, n, top_at=None):
    """Uniform limbs with limb ``top_at`` (default n-1) nonzero and limbs above it zero.

    ``top_at`` may be an array (per-row precision - 1).
    """
    states = np.asarray(states, dtype=np.uint64).reshape(-1)
    x = limbs(states, n)
    rows = np.arange(len(states))
    top = np.full(len(states), n - 1, dtype=np.int64) if top_at is None else np.asarray(top_at, dtype=np.int64)
    cols = np.arange(n)[None, :]
    x = np.where(cols > top[:, None], np.uint32(0), x)
    for r in rows[x[rows, top] == 0]:
        k = n
        while True:
            d = int(draws(states[r:r + 1], k, 1)[0, 0] >> np.uint64(32))
            if d:
                x[r, top[r]] = d
                break
            k += 1
    return x


def uniform_int(states, lo, hi, draw_index=0):
    """Uniform integer in [lo, hi] per generator (multiply-shift on a 64-bit draw)."""
    d = draws(states, draw_index, 1)[:, 0]
    span = np.asarray(hi, dtype=object) - np.asarray(lo, dtype=object) + 1
    out = [int(lo_) + ((int(x) * int(s)) >> 64)
           for x, lo_, s in zip(d, np.broadcast_to(np.asarray(lo, dtype=object), d.shape),
                                np.broadcast_to(span, d.shape))]
    return np.asarray(out, dtype=np.int64)


# ---------------------------------------------------------------- conversions

def to_int(row):
    """Little-endian uint32 limb row -> Python int."""
    return int.from_bytes(np.ascontiguousarray(row, dtype="<u4").tobytes(), "little")


def from_int(x, n):
    """Python int (0 <= x < 2^(32 n)) -> little-endian uint32 limb row of length n."""
    return np.frombuffer(int(x).to_bytes(4 * n, "little"), dtype="<u4").astype(np.uint32)


# ---------------------------------------------------------------- workloads

def random_pairs(seed, batch, nu, nv, nv_eff=None, nu_eff=None):
    """u: nu limbs (top limb nonzero at nu_eff-1), v: nv-limb buffer with top
    nonzero limb at nv_eff-1 (scalar or per-instance array), uniform limbs."""
    st = instance_states(seed, np.arange(batch))
    top_u = None if nu_eff is None else np.broadcast_to(np.asarray(nu_eff) - 1, (batch,))
    top_v = None if nv_eff is None else np.broadcast_to(np.asarray(nv_eff) - 1, (batch,))
    u = limbs_top_nonzero(substream(st, 0), nu, top_u)
    v = limbs_top_nonzero(substream(st, 1), nv, top_v)
    return u, v


def config_c1():
    """2^15-bit division: 1024 instances, u 1024 limbs, v 512 limbs, top limbs nonzero."""
    u, v = random_pairs(SEED_C1, 1024, 1024, 512)
    return {"name": "divrem_2p15_b1024", "u": u, "v": v, "nq": 513, "bits": 1 << 15}


C2_FAMILIES = ("F1 v=B^1024-1", "F2 v=B^1023+1", "F3 v top limb 1",
               "F4 u=v*w+v-1", "F5 u<v")


def c2_family(j):
    """-1 for a uniform-random instance, else the adversarial family index 0..4."""
    return -1 if j % 4 != 3 else (j // 4) % 5


def config_c2(batch=4096, index=None):
    """2^16-bit division: u 2048 limbs, v 1024 limbs; instance j with j mod 4 == 3
    is adversarial with family (j div 4) mod 5 (see ``C2_FAMILIES``).

    ``index`` selects a subset of instance indices (default: all ``batch``)."""
    nu, nv = 2048, 1024
    idx = np.arange(batch) if index is None else np.asarray(index, dtype=np.int64)
    st = instance_states(SEED_C2, idx)
    s0, s1, s2, s3 = (substream(st, t) for t in range(4))
    u = limbs_top_nonzero(s0, nu)
    v = limbs_top_nonzero(s1, nv)
    for r, j in enumerate(idx):
        f = c2_family(int(j))
        if f == 0:                       # v = B^1024 - 1
            v[r, :] = 0xFFFFFFFF
        elif f == 1:                     # v = B^1023 + 1
            v[r, :] = 0
            v[r, 0] = 1
            v[r, nv - 1] = 1
        elif f == 2:                     # top limb of v is 1
            v[r, nv - 1] = 1
        elif f == 3:                     # u = v*w + v - 1, expected (w, v - 1)
            w = limbs_top_nonzero(s3[r:r + 1], nv - 1)[0]
            vi, wi = to_int(v[r]), to_int(w)
            u[r] = from_int(vi * wi + vi - 1, nu)
        elif f == 4:                     # u < v
            lo = limbs(s0[r:r + 1], nv - 1)[0]
            top = int(uniform_int(s2[r:r + 1], 0, int(v[r, nv - 1]) - 1)[0])
            u[r, :] = 0
            u[r, :nv - 1] = lo
            u[r, nv - 1] = top
    return {"name": "divrem_2p16_b4096", "u": u, "v": v, "nq": 1025, "bits": 1 << 16,
            "index": idx}


def config_c3(batch=256, index=None):
    """2^18-bit division: u 8192 limbs; divisor length uniform in [2048, 8192]
    limbs per instance, stored zero-padded in an 8192-limb buffer."""
    n = 8192
    idx = np.arange(batch) if index is None else np.asarray(index, dtype=np.int64)
    st = instance_states(SEED_C3, idx)
    nv_eff = uniform_int(substream(st, 2), 2048, 8192)
    u = limbs_top_nonzero(substream(st, 0), n)
    v = limbs_top_nonzero(substream(st, 1), n, nv_eff - 1)
    return {"name": "divrem_2p18_b256", "u": u, "v": v, "nq": 6145, "bits": 1 << 18,
            "nv_eff": nv_eff, "index": idx}


C4_WIDTHS = (1024, 2048, 4096, 8192)   # 2^15 .. 2^18 bits


def config_c4(count=8192, index=None):
    """Mixed precisions: dividend width uniform over {1024, 2048, 4096, 8192}
    limbs (top limb nonzero), divisor length uniform in [ceil(n/4), n] limbs
    (top limb nonzero).  Returns per-instance lists of u and v rows."""
    idx = np.arange(count) if index is None else np.asarray(index, dtype=np.int64)
    st = instance_states(SEED_C4, idx)
    s2 = substream(st, 2)
    ns = np.asarray(C4_WIDTHS)[uniform_int(s2, 0, 3, draw_index=0)]
    nvs = np.array([int(uniform_int(s2[r:r + 1], (n + 3) // 4, n, draw_index=1)[0]) for r, n in enumerate(ns)])
    s0, s1 = substream(st, 0), substream(st, 1)
    us = [limbs_top_nonzero(s0[r:r + 1], int(n))[0] for r, n in enumerate(ns)]
    vs = [limbs_top_nonzero(s1[r:r + 1], int(nv))[0] for r, nv in enumerate(nvs)]
    return {"name": "divrem_mixed_2p15_2p18_b%d" % len(idx), "u": us, "v": vs, "n": ns, "nv": nvs,
            "index": idx}


def config_c5(rate, count=10000, index=None):
    """Serving workload: request j arrives after exponential gaps of mean
    1/rate seconds (Poisson arrivals); its dividend has n = round(2^x / 32)
    limbs with x uniform in [15, 18] (top limb nonzero) and its divisor a
    length uniform in [ceil(n/8), n] (top limb nonzero).  The operands do not
    depend on the rate; the arrival times do."""
    idx = np.arange(count) if index is None else np.asarray(index, dtype=np.int64)
    st = instance_states(SEED_C5, idx)
    s2 = substream(st, 2)
    x = 15.0 + 3.0 * (draws(s2, 0, 1)[:, 0] >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    ns = np.rint(2.0 ** x / 32.0).astype(np.int64)
    nvs = np.array([int(uniform_int(s2[r:r + 1], (n + 7) // 8, n, draw_index=1)[0]) for r, n in enumerate(ns)])
    s0, s1 = substream(st, 0), substream(st, 1)
    us = [limbs_top_nonzero(s0[r:r + 1], int(n))[0] for r, n in enumerate(ns)]
    vs = [limbs_top_nonzero(s1[r:r + 1], int(nv))[0] for r, nv in enumerate(nvs)]
    arrival = c5_arrivals(rate, int(idx.max()) + 1)[idx] if len(idx) else np.zeros(0)
    return {"name": "serve_2p15_2p18_rate%g_n%d" % (rate, len(idx)), "u": us, "v": vs, "n": ns, "nv": nvs,
            "arrival": arrival, "rate": rate, "index": idx}


def c5_arrivals(rate, count):
    """Arrival times (s) of the first `count` serving requests at `rate` per
    second: cumulative exponential gaps drawn from a generator of their own
    (seeded by the rate), gap = -ln(U) / rate with U uniform in (0, 1)."""
    ga = draws(np.array([np.uint64(SEED_C5 ^ int(rate * 1000))], dtype=np.uint64), 0, count)[0]
    uni = ((ga >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
    return np.cumsum(-np.log(uni) / rate)
