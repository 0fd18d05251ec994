"""The sorting network of Section 7.1 compiled to BMMC passes (Section 7.2):
the host compilation on the CPU, applied stage by stage with the oracle's
permutation, and the device forms against the oracle's sort."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2306_07795_amd import binding as B


def keys(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.integers(-(1 << 31), 1 << 31, size=1 << n, dtype=np.int64).astype(np.int32)
    if n >= 3:
        a[rng.integers(0, 1 << n, size=(1 << n) // 4)] = a[0]  # duplicates
        a[1] = np.int32(-1)
        a[2] = np.int32(0x7FFFFFFF)
    return a


def cmpx_pairs(a, signed):
    v = a.view(np.int32 if signed else np.uint32).reshape(-1, 2)
    lo, hi = np.minimum(v[:, 0], v[:, 1]), np.maximum(v[:, 0], v[:, 1])
    return np.stack([lo, hi], axis=1).reshape(-1).view(a.dtype)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 6, 12, 20, 32])
def test_stage_count_and_product(n):
    st = B.bmmc_sortnet_stages(n)
    assert len(st) == n * (n + 1) // 2 + 1
    prod = np.eye(n, dtype=np.uint8)
    for rows in st:
        m = O.dense(rows, n)
        assert O.rank(m) == n
        prod = O.mul(m, prod)
    assert np.array_equal(prod, np.eye(n, dtype=np.uint8))


@pytest.mark.parametrize("signed", [True, False])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 10])
def test_compiled_network_sorts_on_the_cpu(n, signed):
    """Every stage applied with the oracle's permutation, every column as
    pairwise min/max of adjacent keys: the oracle's sort."""
    a = keys(n, n)
    st = B.bmmc_sortnet_stages(n)
    x = a
    for s, rows in enumerate(st):
        x = O.permute(x, n, rows, 0)
        if s + 1 < len(st):
            x = cmpx_pairs(x, signed)
    assert np.array_equal(x, O.sort_keys(a, signed))


@pytest.mark.parametrize("signed", [True, False])
@pytest.mark.parametrize("n", [2, 3, 5, 8, 12, 13, 14, 16, 18])
def test_fused_passes_sort_on_the_cpu(n, signed):
    """The device passes (stages grouped, columns in LDS) emulated on the host
    with the kernel's own tables: the oracle's sort, in far fewer passes than
    columns, and in one pass while the array fits one tile."""
    a = keys(n, 7 * n + signed)
    out = np.zeros_like(a)
    passes = B.bmmc_sortnet_emulate(a, out, n, B.KEY_I32 if signed else B.KEY_U32)
    assert np.array_equal(out, O.sort_keys(a, signed))
    assert B.bmmc_sortnet_passes(n)[0] == passes
    columns = n * (n + 1) // 2
    assert passes <= columns + 1
    if n <= 13:
        assert passes == 1
    else:
        assert passes < columns // 3


def test_errors():
    with pytest.raises(B.BmmcError):
        B.bmmc_sortnet_stages(33)


# ------------------------------------------------------------------ device

def run_device(a, n, signed, method):
    from tests import gpu_util as G
    x = G.to_device(a)
    y = G.empty_like_bytes(a)
    B.bmmc_sortnet(x, y, n, B.KEY_I32 if signed else B.KEY_U32, method, G.stream())
    G.sync()
    assert np.array_equal(G.to_host(x, a), a)  # the input is left alone
    return G.to_host(y, a)


@pytest.mark.gpu
@pytest.mark.parametrize("method", [B.SORTNET_PASSES, B.SORTNET_DIRECT])
@pytest.mark.parametrize("signed", [True, False])
@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 8, 11, 12, 13, 14, 17, 20])
def test_device_network_equals_oracle_sort(n, signed, method):
    a = keys(n, 100 + n)
    assert np.array_equal(run_device(a, n, signed, method), O.sort_keys(a, signed))


@pytest.mark.gpu
@pytest.mark.parametrize("method", [B.SORTNET_PASSES, B.SORTNET_DIRECT])
@pytest.mark.parametrize("kind", ["sorted", "reversed", "equal", "two_values"])
def test_device_network_special_inputs(kind, method):
    n = 15
    base = np.arange(-(1 << 14), 1 << 14, dtype=np.int32)
    a = {"sorted": base, "reversed": base[::-1].copy(), "equal": np.full(1 << n, 7, np.int32),
         "two_values": np.where(np.arange(1 << n) % 3 == 0, -5, 9).astype(np.int32)}[kind]
    assert np.array_equal(run_device(a, n, True, method), O.sort_keys(a, True))


@pytest.mark.gpu
@pytest.mark.parametrize("method", [B.SORTNET_PASSES, B.SORTNET_DIRECT])
def test_device_network_2p24_full(method):
    """2^24 int32 keys (the largest size the benchmark sorts), in full."""
    n = 24
    a = keys(n, 24)
    assert np.array_equal(run_device(a, n, True, method), O.sort_keys(a, True))
