"""Writer of the ``.pyromech`` version-1 mechanism file.

Layout (little endian).  A 48-byte header::

    0  char[8] "PYROMECH"      24 u32 n_third_body (class 1)
    8  u32 version = 1         28 u32 n_falloff (classes 2 and 3)
    12 u32 S  (species)        32 u32 nnz of the reactant lists
    16 u32 R  (reactions)      36 u32 nnz of the product lists
    20 u32 E  (elements)       40 u64 payload bytes

then the payload, each array zero-padded to a multiple of 8 bytes::

    f64 element_weight[E]            kg/mol
    i32 composition[E][S]            atoms of element e in species k
    f64 W[S]                         kg/mol
    f64 T_range[S][3]                T_low, T_mid, T_high (K)
    f64 nasa[S][2][7]                low range a1..a7, high range a1..a7
    i32 rtype[R]                     0 elementary, 1 third-body,
                                     2 Lindemann falloff, 3 Troe falloff
    i32 reversible[R]
    f64 arrhenius[R][3]              ln A (SI), b, Ea (J/mol)
    i32 reac_ptr[R+1], reac_species[nnz], reac_nu[nnz]
    i32 prod_ptr[R+1], prod_species[nnz], prod_nu[nnz]
    i32 falloff_reaction[n_falloff]  increasing reaction index
    f64 falloff_low[n_falloff][3]    low-pressure ln A, b, Ea
    f64 troe[n_falloff][4]           alpha, T***, T*, T** (ignored for class 2)
    f64 efficiency[n_tb+n_falloff][S] rows follow the reactions of class >= 1
                                     in increasing index

and a trailing u64 FNV-1a hash of every preceding byte.
"""

import struct

import numpy as np

MAGIC = b"PYROMECH"
VERSION = 1
HEADER = struct.Struct("<8sIIIIIIIIQ")
FNV_OFFSET = 0xcbf29ce484222325
FNV_PRIME = 0x100000001b3


def fnv1a64(data: bytes) -> int:
    """64-bit FNV-1a, vectorised over 8-byte words is not the definition, so
    this folds bytes one at a time (fast enough for files of a few MB)."""
    h = FNV_OFFSET
    mask = (1 << 64) - 1
    for b in data:
        h ^= b
        h = (h * FNV_PRIME) & mask
    return h


def _pad8(b: bytes) -> bytes:
    return b + b"\0" * (-len(b) % 8)


def write(path, *, element_weight, composition, W, T_range, nasa, rtype,
          reversible, arrhenius, reactants, products, falloff_low, troe,
          efficiency):
    """Serialise a mechanism.

    ``reactants``/``products`` are lists (one per reaction) of
    ``(species, nu)`` pairs with integer nu >= 1.  ``falloff_low`` and
    ``troe`` follow the falloff reactions (class 2 or 3) in index order and
    ``efficiency`` the reactions of class >= 1 in index order.
    """
    E, S = composition.shape
    R = len(rtype)
    rtype = np.asarray(rtype, dtype=np.int32)
    n_tb = int((rtype == 1).sum())
    n_fo = int(((rtype == 2) | (rtype == 3)).sum())

    def csr(sides):
        ptr = [0]
        sp, nu = [], []
        for side in sides:
            for k, v in side:
                sp.append(int(k))
                nu.append(int(v))
            ptr.append(len(sp))
        return (np.array(ptr, np.int32), np.array(sp, np.int32),
                np.array(nu, np.int32))

    rp, rs, rn = csr(reactants)
    pp, ps, pn = csr(products)
    fo_rxn = np.nonzero((rtype == 2) | (rtype == 3))[0].astype(np.int32)
    parts = [
        np.asarray(element_weight, np.float64).reshape(E),
        np.asarray(composition, np.int32).reshape(E, S),
        np.asarray(W, np.float64).reshape(S),
        np.asarray(T_range, np.float64).reshape(S, 3),
        np.asarray(nasa, np.float64).reshape(S, 2, 7),
        rtype,
        np.asarray(reversible, np.int32).reshape(R),
        np.asarray(arrhenius, np.float64).reshape(R, 3),
        rp, rs, rn, pp, ps, pn,
        fo_rxn,
        np.asarray(falloff_low, np.float64).reshape(n_fo, 3),
        np.asarray(troe, np.float64).reshape(n_fo, 4),
        np.asarray(efficiency, np.float64).reshape(n_tb + n_fo, S),
    ]
    payload = b"".join(_pad8(np.ascontiguousarray(a).astype(a.dtype.newbyteorder("<")).tobytes())
                       for a in parts)
    head = HEADER.pack(MAGIC, VERSION, S, R, E, n_tb, n_fo, len(rs), len(ps),
                       len(payload))
    body = head + payload
    with open(path, "wb") as f:
        f.write(body)
        f.write(struct.pack("<Q", fnv1a64(body)))
