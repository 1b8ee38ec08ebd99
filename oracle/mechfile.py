"""Reader of the ``.pyromech`` version-1 mechanism file (oracle side).

An independent parser: it shares no code with the GPU library's loader or with
the writer.  The layout is a 48-byte header (magic ``PYROMECH``, u32 version,
S, R, E, n_third_body, n_falloff, reactant nnz, product nnz, u64 payload
bytes), the payload arrays each padded to 8 bytes, and a trailing u64 FNV-1a
hash of all preceding bytes.
"""

import struct
from dataclasses import dataclass

import numpy as np


class MechanismFileError(ValueError):
    pass


@dataclass
class Mechanism:
    """Mechanism data in the paper's notation.

    ``nu_f[k, j]`` = nu'_kj and ``nu_r[k, j]`` = nu''_kj (eq. reactions);
    ``arrhenius[j]`` = (ln A_j, b_j, Ea_j) with Ea in J/mol (eq. rate_coeff,
    theta_a = Ea / R); ``efficiency[i]`` holds the third-body efficiencies of
    reaction ``pd_reactions[i]``; ``falloff_low[f]`` and ``troe[f]`` belong to
    reaction ``falloff_reactions[f]``.
    """
    S: int
    R: int
    E: int
    element_weight: np.ndarray
    composition: np.ndarray   # (E, S)
    W: np.ndarray             # (S,)
    T_range: np.ndarray       # (S, 3)
    nasa_low: np.ndarray      # (S, 7)
    nasa_high: np.ndarray     # (S, 7)
    rtype: np.ndarray         # (R,)
    reversible: np.ndarray    # (R,)
    arrhenius: np.ndarray     # (R, 3)
    nu_f: np.ndarray          # (S, R)
    nu_r: np.ndarray          # (S, R)
    falloff_reactions: np.ndarray
    falloff_low: np.ndarray   # (n_fo, 3)
    troe: np.ndarray          # (n_fo, 4)
    pd_reactions: np.ndarray
    efficiency: np.ndarray    # (n_pd, S)

    @property
    def nu(self):
        """Net stoichiometric coefficients nu = nu'' - nu' (eq. production_rates)."""
        return self.nu_r - self.nu_f

    @property
    def T_mid(self):
        return self.T_range[:, 1]

    @property
    def n_falloff(self):
        return len(self.falloff_reactions)

    def parameters(self):
        """Arrhenius triples in the order the gradients use: the R main
        triples, then the low-pressure triples of the falloff reactions."""
        return np.concatenate([self.arrhenius, self.falloff_low], axis=0)


def _fnv1a64(data: bytes) -> int:
    h = 0xcbf29ce484222325
    for byte in data:
        h = ((h ^ byte) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return h


def load(path) -> Mechanism:
    with open(path, "rb") as f:
        blob = f.read()
    return parse(blob)


def parse(blob: bytes) -> Mechanism:
    if len(blob) < 56:
        raise MechanismFileError("file too short")
    magic, version, S, R, E, n_tb, n_fo, nnz_r, nnz_p, nbytes = \
        struct.unpack_from("<8sIIIIIIIIQ", blob, 0)
    if magic != b"PYROMECH":
        raise MechanismFileError("bad magic")
    if version != 1:
        raise MechanismFileError(f"unknown version {version}")
    if len(blob) != 48 + nbytes + 8:
        raise MechanismFileError("size does not match the header")
    (stored,) = struct.unpack_from("<Q", blob, 48 + nbytes)
    if stored != _fnv1a64(blob[:48 + nbytes]):
        raise MechanismFileError("checksum mismatch")

    pos = [48]

    def take(dtype, count):
        dt = np.dtype(dtype).newbyteorder("<")
        size = dt.itemsize * count
        a = np.frombuffer(blob, dtype=dt, count=count, offset=pos[0]).astype(dt.newbyteorder("="))
        pos[0] += size + (-size % 8)
        return a

    ew = take("f8", E)
    comp = take("i4", E * S).reshape(E, S)
    W = take("f8", S)
    T_range = take("f8", S * 3).reshape(S, 3)
    nasa = take("f8", S * 14).reshape(S, 2, 7)
    rtype = take("i4", R)
    rev = take("i4", R)
    arrh = take("f8", R * 3).reshape(R, 3)
    rp = take("i4", R + 1)
    rs = take("i4", nnz_r)
    rn = take("i4", nnz_r)
    pp = take("i4", R + 1)
    ps = take("i4", nnz_p)
    pn = take("i4", nnz_p)
    fo = take("i4", n_fo)
    low = take("f8", n_fo * 3).reshape(n_fo, 3)
    troe = take("f8", n_fo * 4).reshape(n_fo, 4)
    eff = take("f8", (n_tb + n_fo) * S).reshape(n_tb + n_fo, S)
    if pos[0] != 48 + nbytes:
        raise MechanismFileError("payload size mismatch")

    nu_f = np.zeros((S, R))
    nu_r = np.zeros((S, R))
    for j in range(R):
        for q in range(rp[j], rp[j + 1]):
            nu_f[rs[q], j] += rn[q]
        for q in range(pp[j], pp[j + 1]):
            nu_r[ps[q], j] += pn[q]
    pd = np.nonzero(rtype >= 1)[0]
    return Mechanism(S=S, R=R, E=E, element_weight=ew, composition=comp, W=W,
                     T_range=T_range, nasa_low=nasa[:, 0, :].copy(),
                     nasa_high=nasa[:, 1, :].copy(), rtype=rtype,
                     reversible=rev, arrhenius=arrh, nu_f=nu_f, nu_r=nu_r,
                     falloff_reactions=fo, falloff_low=low, troe=troe,
                     pd_reactions=pd, efficiency=eff)
