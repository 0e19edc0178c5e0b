"""Host-side tools that need no GPU: the multi-step history comparison and
the benchmark's radix pass count."""
import json
import subprocess
import sys

import numpy as np


def test_multistep_compare(tmp_path):
    # two histories of the conserved sums (rows: E_kin, E_int, E_pot, E,
    # P[3], L[3]); the second's energy is offset by 1e-8 at every step and
    # drifts by an extra 2e-10 per step, its momentum by 3e-14 at the last
    k = 6
    a = np.zeros((k, 10))
    a[:, 3] = -0.5 + 1e-9 * np.arange(k)
    b = a.copy()
    b[:, 3] += 1e-8 + 2e-10 * np.arange(k)
    b[-1, 4] += 3e-14
    pa, pb = tmp_path / "a.npy", tmp_path / "b.npy"
    np.save(pa, a)
    np.save(pb, b)
    out = subprocess.run([sys.executable, "-m", "paper_1807_08116_amd.multistep", "--compare",
                          str(pa), str(pb)], capture_output=True, text=True, check=True)
    r = json.loads(out.stdout)
    assert r["steps_compared"] == k - 1
    E0 = abs(b[0, 3])
    np.testing.assert_allclose(r["energy_gap_max"], (1e-8 + 2e-10 * (k - 1)) / E0, rtol=1e-6)
    np.testing.assert_allclose(r["energy_change_gap_max"], 2e-10 * (k - 1) / E0, rtol=1e-6)
    np.testing.assert_allclose(r["momentum_gap_max"], 3e-14, rtol=1e-6)
    assert r["angmom_gap_max"] == 0.0


def test_radix_pass_count():
    # 10-bit digits: cell keys below cell_cap need ceil(bits / 10) passes
    import bench
    assert bench.radix_passes(1) == 1
    assert bench.radix_passes(1024) == 1            # keys 0 .. 1023: 10 bits
    assert bench.radix_passes(1025) == 2
    assert bench.radix_passes(1 << 20) == 2
    assert bench.radix_passes((1 << 20) + 1) == 3
    assert bench.radix_passes(8 * 1048576 + 4096) == 3   # the c2 default capacity
