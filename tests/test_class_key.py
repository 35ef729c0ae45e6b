"""The class key of Sec. 3.2: the 64-bit FNV-1a hash of a fault's signature.

On the CPU, the FNV-1a used here is pinned to the published test vectors of
the 64-bit variant, and its vectorised form to the plain byte loop. On the
GPU, the keys the hash kernel writes for every fault position (copied by a
test hook before the grouping passes reuse that buffer) must equal, as a
multiset, the FNV-1a hashes of the oracle's per-fault signatures laid out as
the compiler lays out a signature: ceil(D/64) detector words, then
ceil(O/64) observable words, each word's octets little-endian, the hash cut to
the key bits the compile keeps.
"""

import sys

import numpy as np
import pytest

import oracle
from paper_2604_16613_amd import Driver
from paper_2604_16613_amd import _gp
from workloads import (bit_flip_code_fig1, bivariate_bicycle_memory, log_uniform_rates, mirror_circuit,
                       repetition_code_memory, rotated_surface_code_memory)

FNV_OFFSET = 0xcbf29ce484222325
FNV_PRIME = 0x100000001b3
M64 = (1 << 64) - 1


def fnv1a64(data: bytes) -> int:
    """FNV-1a, 64 bits: for each octet, xor it in, then multiply by the prime."""
    h = FNV_OFFSET
    for o in data:
        h = ((h ^ o) * FNV_PRIME) & M64
    return h


def fnv1a64_words(words: np.ndarray) -> np.ndarray:
    """FNV-1a over the little-endian octets of each row of a (F, W) uint64
    array, vectorised over the rows (uint64 arithmetic wraps mod 2^64)."""
    f = words.shape[0]
    h = np.full(f, FNV_OFFSET, dtype=np.uint64)
    p = np.uint64(FNV_PRIME)
    with np.errstate(over="ignore"):
        for w in range(words.shape[1]):
            col = words[:, w]
            for o in range(8):
                h = (h ^ ((col >> np.uint64(8 * o)) & np.uint64(0xff))) * p
    return h


def signature_words(res) -> np.ndarray:
    """(F, W) signature words of every fault of an oracle result (keep_faults)."""
    d, o = res.n_detectors, res.n_observables
    wd = (d + 63) // 64
    w = wd + (o + 63) // 64
    f = res.n_faults
    out = np.zeros((f, w), dtype=np.uint64)
    bits = res.fault_bits.astype(np.int64)
    owner = np.repeat(np.arange(f), np.diff(res.fault_off))
    is_obs = bits >= d
    word = np.where(is_obs, wd + (bits - d) // 64, bits // 64)
    bit = np.where(is_obs, (bits - d) % 64, bits % 64).astype(np.uint64)
    np.bitwise_or.at(out, (owner, word), np.left_shift(np.uint64(1), bit))
    return out


def test_fnv1a64_published_vectors():
    assert fnv1a64(b"") == 0xcbf29ce484222325
    assert fnv1a64(b"a") == 0xaf63dc4c8601ec8c
    assert fnv1a64(b"foobar") == 0x85944171f73967e8


def test_vectorised_hash_equals_byte_loop():
    rng = np.random.default_rng(7)
    for w in (0, 1, 3, 13):
        words = rng.integers(0, 2**63, size=(40, w), dtype=np.uint64)
        words[::3] = 0  # all-zero signatures
        if w:
            words[1::4, -1] = np.uint64(1) << np.uint64(63)  # a lone top bit
        got = fnv1a64_words(words)
        for r in range(words.shape[0]):
            assert int(got[r]) == fnv1a64(words[r].astype("<u8").tobytes())


def test_signature_layout():
    """Detector d in word d // 64, observable k in word ceil(D/64) + k // 64."""
    class R:
        n_detectors, n_observables, n_faults = 70, 2, 3
        fault_off = np.array([0, 2, 2, 4])
        fault_bits = np.array([0, 69, 70, 71])
    w = signature_words(R)
    assert w.shape == (3, 3)
    assert list(w[0]) == [1, 1 << 5, 0]
    assert list(w[1]) == [0, 0, 0]
    assert list(w[2]) == [0, 0, 0b11]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


CASES = [
    ("fig1", lambda: (bit_flip_code_fig1().text, None)),
    ("rep7", lambda: (repetition_code_memory(7, 5, p_data=0.01, p_meas=0.02, p2=0.03, p1=0.04).text, None)),
    ("mirror", lambda: (mirror_circuit(5, 6, 2, x_basis=[2, 3]).text, None)),
    ("sc5", lambda: (rotated_surface_code_memory(5, 5).text, None)),
    ("sc11 rates", lambda: (lambda c: (c.text, log_uniform_rates(c.n_channels, 2)))(rotated_surface_code_memory(11, 11))),
    ("bb r3", lambda: (bivariate_bicycle_memory(rounds=3).text, None)),
    ("sc17", lambda: (rotated_surface_code_memory(17, 17).text, None)),
]


@pytest.fixture(scope="module")
def key_driver():
    say("creating a driver for d=17 r=17 and the [[144,12,12]] code, key capture on")
    b = _gp.gp_bounds_from_circuit(rotated_surface_code_memory(17, 17).text)
    bb = _gp.gp_bounds_from_circuit(bivariate_bicycle_memory(rounds=3).text)
    for k, _ in b._fields_:
        setattr(b, k, max(getattr(b, k), getattr(bb, k)))
    b.max_slab_words = 0
    b.max_items = 0
    d = Driver(b)
    _gp.gp_debug_capture_keys(d.handle, True)
    yield d
    _gp.gp_debug_capture_keys(d.handle, False)
    d.close()


def check_keys(drv, text, rates, label):
    say("case", label)
    drv.compile_hypergraph(text, rates)
    keys, bits = _gp.gp_debug_class_keys(drv.handle)
    res = oracle.run(text, rates=rates, keep_faults=True, threads=8)
    assert len(keys) == res.n_faults, label
    mask = np.uint64(M64 if bits >= 64 else (1 << bits) - 1)
    want = fnv1a64_words(signature_words(res)) & mask
    assert np.array_equal(np.sort(keys), np.sort(want)), f"{label}: device keys are not FNV-1a of the signatures"
    return bits


@pytest.mark.gpu
@pytest.mark.parametrize("name", [c[0] for c in CASES])
def test_device_keys_are_fnv1a_of_signatures(key_driver, name):
    text, rates = dict(CASES)[name]()
    bits = check_keys(key_driver, text, rates, name)
    assert 16 <= bits <= 64


@pytest.mark.gpu
def test_device_keys_cut_to_forced_bits(key_driver):
    """With the key cut to 12 bits by the test hook, the captured keys are the
    low 12 bits of the same hashes (the compile then re-runs keyed on both
    hashes, which the capture does not see)."""
    _gp.gp_debug_set_key_bits(key_driver.handle, 12)
    try:
        bits = check_keys(key_driver, rotated_surface_code_memory(5, 5).text, None, "sc5, 12 key bits")
    finally:
        _gp.gp_debug_set_key_bits(key_driver.handle, 64)
    assert bits == 12


@pytest.mark.gpu
def test_batch_keys_salted_after_the_first_circuit():
    """In a batch the first circuit's positions carry the plain FNV-1a keys of
    its signatures; a later circuit's keys carry a per-circuit salt, so even an
    identical circuit in the second slot gets other keys (classes are never
    merged across circuits)."""
    c = rotated_surface_code_memory(5, 5).text
    say("batch of two identical d=5 circuits, key capture on")
    d = Driver.from_batch([c, c])
    try:
        _gp.gp_debug_capture_keys(d.handle, True)
        d.compile_batch([c, c])
        keys, bits = _gp.gp_debug_class_keys(d.handle)
    finally:
        d.close()
    res = oracle.run(c, keep_faults=True)
    f0 = res.n_faults
    assert len(keys) == 2 * f0
    mask = np.uint64(M64 if bits >= 64 else (1 << bits) - 1)
    want = np.sort(fnv1a64_words(signature_words(res)) & mask)
    assert np.array_equal(np.sort(keys[:f0]), want)
    assert not np.array_equal(np.sort(keys[f0:]), want)
    assert len(np.intersect1d(keys[:f0], keys[f0:])) == 0
