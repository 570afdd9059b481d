"""GPU check of the matrix-core rate probe (dsrg_df_mfma_probe), the
measurement aid behind the bench's sustained-rate figures: on a tiny launch
the int8 probe's folded sums equal a host evaluation of the products it is
meant to take (so the timed launches really run iters x 8 products of the
stated shape per wave), the FP64 probe is finite and repeatable, and the
per-workgroup counter stamps advance."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
M64 = (1 << 64) - 1


def _b():
    from paper_1603_00561_amd import binding
    return binding


def mix(z):
    """splitmix64 finalizer on python ints (Steele, Lea and Flood, 2014)."""
    z = (z + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def operand_bytes(gid, base):
    """The 16 int8 values of one i4v operand: four int32 words (low 32 bits of
    the mixed index), little-endian."""
    words = np.array([mix(gid * 64 + base + e) & 0xFFFFFFFF for e in range(4)], dtype=np.uint32)
    return words.view(np.int8)


def expected_i8_sink(nwg, iters):
    out = np.zeros(nwg * 512, dtype=np.uint32)
    for w in range(nwg * 8):
        gids = [w * 64 + l for l in range(64)]
        A = np.zeros((8, 32, 32), np.int64)   # [m][row][k]
        B = np.zeros((8, 32, 32), np.int64)   # [m][k][col]
        for lane, g in enumerate(gids):
            for m in range(8):
                A[m, lane % 32, 16 * (lane // 32):16 * (lane // 32) + 16] = operand_bytes(g, m * 8)
                B[m, 16 * (lane // 32):16 * (lane // 32) + 16, lane % 32] = operand_bytes(g, m * 8 + 4)
        acc = np.zeros((4, 32, 32), np.int64)
        for m in range(8):
            acc[m & 3] += A[m] @ B[(3 * m + 1) & 7]
        acc = (acc * iters) % (1 << 32)
        for lane, g in enumerate(gids):
            r = np.arange(16)
            rows = 8 * (r // 4) + 4 * (lane // 32) + r % 4
            out[g] = np.uint32(int(acc[:, rows, lane % 32].sum()) % (1 << 32))
    return out


def _run(kind, nwg, iters):
    dev = torch.device("cuda:0")
    stamps = torch.zeros(4 * nwg, dtype=torch.int64, device=dev)
    sink = torch.zeros(512 * nwg, dtype=torch.int32 if kind == "i8" else torch.float64,
                       device=dev)
    print(f"[gpu-probe] kind={kind} nwg={nwg} iters={iters}", flush=True)
    _b().mfma_probe(kind, nwg, iters, stamps, sink)
    torch.cuda.synchronize()
    return stamps.view(nwg, 4).cpu().numpy(), sink.cpu().numpy()


def test_i8_probe_takes_the_stated_products():
    nwg, iters = 2, 5
    st, sink = _run("i8", nwg, iters)
    assert np.array_equal(sink.view(np.uint32), expected_i8_sink(nwg, iters))
    assert (st[:, 2] > st[:, 0]).all() and (st[:, 3] >= st[:, 1]).all()


def test_f64_probe_is_finite_and_repeatable():
    st1, s1 = _run("f64", 4, 16)
    st2, s2 = _run("f64", 4, 16)
    assert np.isfinite(s1).all() and np.array_equal(s1, s2) and np.abs(s1).max() > 0
    assert (st1[:, 2] > st1[:, 0]).all() and (st1[:, 3] >= st1[:, 1]).all()


def test_probe_rejects_bad_buffers():
    b = _b()
    dev = torch.device("cuda:0")
    stamps = torch.zeros(8, dtype=torch.int64, device=dev)
    with pytest.raises(ValueError):
        b.mfma_probe("i8", 4, 1, stamps, torch.zeros(4 * 512, dtype=torch.int32, device=dev))
    with pytest.raises(ValueError):
        b.mfma_probe("f64", 2, 1, stamps, torch.zeros(2 * 512, dtype=torch.int32, device=dev))
