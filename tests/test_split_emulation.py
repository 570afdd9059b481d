"""CPU emulation of the two split-precision schemes for the (ia|jb)
contractions, against the FP64 oracle: the reason the library builds
error-free int8 slices and not the BF16 hi/lo scheme.

* BF16 x3: B = hi + lo with hi = bf16(B), lo = bf16(B - hi) (round to
  nearest even, emulated by integer rounding of the float32 bit pattern), the
  three products hi.hi + hi.lo + lo.hi accumulated in float32 (numpy sgemm:
  the accumulation order differs from the matrix cores', the rounding unit is
  the same), converted to FP64 before the regulariser and the energy sums.
* int8 slices (Ozaki, Ogita, Oishi and Rump, 2012): per column of B (a vector
  over the auxiliary index) a power-of-two scale sigma >= max |B|, then four
  round-to-nearest slices of x = B / sigma, x ~ (s0 + s1/254 + s2/254^2 +
  s3/254^3) / 127 with |s_k| <= 127; the ten slice products of levels
  k + l <= 3 are exact integer sums (taken here in FP64 BLAS, exact because
  every partial sum stays below 2^53), recombined in FP64 with weights
  sigma_a sigma_b / (127^2 254^(k+l)); the self-pair diagonal (ia|ia) is taken
  in FP64.

Gate of the split path: |dE| <= 1e-6 Eh per term. The emulation shows the
BF16 x3 scheme missing it by orders of magnitude on the triple-zeta-shaped
workload while the int8 slices meet it; it prints |dE| per term for both.
"""
import numpy as np
import pytest

from oracle import dsrg_oracle as O
from paper_1603_00561_amd.workloads import make_config

GATE = 1e-6


def bf16_round(x):
    """Round FP64 values to the nearest BF16 (ties to even), returned as float32."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def bf16x3_prep(B):
    """hi, lo of a block B[Q][a] (float32 arrays holding BF16 values)."""
    hi = bf16_round(B)
    lo = bf16_round(B - hi.astype(np.float64))
    return np.ascontiguousarray(hi.T), np.ascontiguousarray(lo.T), hi, lo


def bf16x3_K(oi, oj, same=False):
    """K[a, b] = sum_Q Bi[Q, a] Bj[Q, b] from three BF16 products, float32 sums."""
    K = oi[0] @ oj[2]
    K = K + oi[0] @ oj[3]
    K = K + oi[1] @ oj[2]
    return K.astype(np.float64)


def int8_slices(B):
    """Scales sigma [ncol] and slices s[4][naux][ncol] (integer-valued FP64)."""
    m = np.abs(B).max(axis=0)
    sig = np.where(m > 0, 2.0 ** np.ceil(np.log2(np.where(m > 0, m, 1.0))), 1.0)
    r = 127.0 * B / sig
    s = []
    for k in range(4):
        sk = np.rint(r)
        s.append(sk)
        r = 254.0 * (r - sk)
    return sig, s


def int8_prep(B):
    """Scales, the slices of each level stacked along Q for the left operand
    ([s0 .. sL]) and the right one ([sL .. s0]), and the FP64 column sums of
    squares (the self-pair diagonal)."""
    sig, S = int8_slices(B)
    left = [np.ascontiguousarray(np.concatenate(S[:L + 1], axis=0).T) for L in range(4)]
    right = [np.ascontiguousarray(np.concatenate(S[L::-1], axis=0)) for L in range(4)]
    return sig, left, right, np.sum(B * B, axis=0)


def int8_K(oi, oj, same=False):
    K = np.zeros((oi[0].size, oj[0].size))
    for L in range(4):
        K += (oi[1][L] @ oj[2][L]) / (127.0 ** 2 * 254.0 ** L)   # exact integer sums
    K *= oi[0][:, None] * oj[0][None, :]
    if same:
        np.fill_diagonal(K, oi[3])
    return K


def ccvv_energy(p, scheme):
    prep, Kf = SCHEMES[scheme]
    naux, nc, nv = p.B_cv.shape
    ops = [prep(np.ascontiguousarray(p.B_cv[:, i, :])) for i in range(nc)]
    parts = []
    for i in range(nc):
        for j in range(i, nc):
            K = Kf(ops[i], ops[j], i == j)
            D = p.eps_c[i] + p.eps_c[j] - p.eps_v[:, None] - p.eps_v[None, :]
            e = float(np.sum(K * (2.0 * K - K.T) * O.reg_R(D, p.s)))
            parts.append(e if i == j else 2.0 * e)
    return float(np.sum(parts))


def cavv_energy(p, scheme):
    prep, Kf = SCHEMES[scheme]
    naux, nc, nv = p.B_cv.shape
    na = p.na
    opc = [prep(np.ascontiguousarray(p.B_cv[:, m, :])) for m in range(nc)]
    opa = [prep(np.ascontiguousarray(p.B_av[:, u, :])) for u in range(na)]
    parts = []
    for m in range(nc):
        X = [Kf(opc[m], opa[u]) for u in range(na)]
        D = [p.eps_c[m] + p.eps_a[u] - p.eps_v[:, None] - p.eps_v[None, :] for u in range(na)]
        for u in range(na):
            Z = X[u] * O.reg_S(D[u], p.s)
            for v in range(na):
                Y = (2.0 * X[v] - X[v].T) * O.reg_R1(D[v], p.s)
                parts.append(p.gamma1[u, v] * float(np.sum(Z * Y)))
    return float(np.sum(parts))


SCHEMES = {"bf16x3": (bf16x3_prep, bf16x3_K), "int8x10": (int8_prep, int8_K)}


def test_bf16_rounding_is_round_to_nearest_even():
    # exact BF16 values survive; halfway cases go to the even mantissa
    x = np.array([1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 0.0])
    want = np.array([1.0, 1.0 + 2 ** -7, 1.0, 1.0 + 2 ** -6, -2.5, 0.0], dtype=np.float32)
    assert np.array_equal(bf16_round(x), want)


def test_int8_slices_reconstruct_to_four_slice_precision():
    rng = np.random.default_rng(3)
    B = rng.standard_normal((200, 17)) * 0.05
    sig, s = int8_slices(B)
    assert all(np.abs(x).max() <= 127 for x in s)
    rec = sig * (s[0] + s[1] / 254 + s[2] / 254 ** 2 + s[3] / 254 ** 3) / 127
    assert np.abs(rec - B).max() <= sig.max() / (127 * 2 * 254 ** 3)


@pytest.mark.parametrize("name", ["cfg1", "cfg2"])
def test_split_schemes_against_the_fp64_oracle(name):
    p = make_config(name)
    ref = {"ccvv": O.energy_ccvv(p.B_cv, p.eps_c, p.eps_v, p.s)}
    if name != "cfg1":
        ref["cavv"] = O.energy_cavv(p.B_cv, p.B_av, p.eps_c, p.eps_a, p.eps_v, p.gamma1, p.s)
    err = {}
    for scheme in SCHEMES:
        err[scheme] = {"ccvv": abs(ccvv_energy(p, scheme) - ref["ccvv"])}
        if "cavv" in ref:
            err[scheme]["cavv"] = abs(cavv_energy(p, scheme) - ref["cavv"])
    print(f"[split-emulation] {name} |dE| (Eh) per term: {err}; |E| {ref}", flush=True)
    # the int8 slices meet the gate on every term
    assert all(v <= GATE for v in err["int8x10"].values()), err
    if name == "cfg2":
        # BF16 x3 misses it on the triple-zeta-shaped workload, by far
        assert err["bf16x3"]["ccvv"] > 100 * GATE, err
