"""The benchmark's byte accounting (CPU only): per-op algorithmic bytes at
N = 2^16, L = 36, k = 12, beta = 3 against the figures derived from the
paper's Table III shapes (key-switch 103.8 MB, HMult 132.1 MB, HRot 113.2 MB,
1 MB = 10^6 B, a limb = 2^18 B), the dominant kernel's bytes, and the rule
that a stored HBM-traffic figure is dropped once the kernel sources change."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


LIMB = 4 * (1 << 16)


def test_per_op_bytes_match_the_derived_figures(bench):
    L, k, beta = 36, 12, 3
    assert round(bench._op_limbs("KEYSWITCH", L, k, beta) * LIMB / 1e6, 1) == 103.8
    assert round(bench._op_limbs("HMULT", L, k, beta) * LIMB / 1e6, 1) == 132.1
    assert round(bench._op_limbs("HROT", L, k, beta) * LIMB / 1e6, 1) == 113.2
    # rescale reads the ciphertext and writes one limb fewer per component
    assert bench._op_limbs("RESCALE", L, k, beta) == 2 * L + 2 * (L - 1)


def test_dominant_kernel_bytes(bench):
    # K5: beta (L + k) ModUp limbs + 2 beta (L + k) key limbs in, 2 (L + k) out
    L, k, beta = 36, 12, 3
    assert (3 * beta + 2) * (L + k) == 528
    assert round(528 * LIMB / 1e6, 1) == 138.4


def test_stored_traffic_needs_the_same_kernel_sources(bench, tmp_path, monkeypatch):
    f = tmp_path / "traffic.txt"
    f.write_text("kernel: k\nbytes_per_launch: 123\nsource_sha256: %s\n" % bench.kernel_source_hash())
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.stored_traffic() == 123
    f.write_text("kernel: k\nbytes_per_launch: 123\nsource_sha256: %s\n" % ("0" * 64))
    assert bench.stored_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.stored_traffic() is None

