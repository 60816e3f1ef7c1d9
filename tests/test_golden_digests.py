"""The oracle digest fixture of the wide-k GPU parity tests is present and
covers exactly the cases its generating script lists (CPU only)."""
import importlib.util
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def test_wide_k_digest_file_matches_its_script():
    spec = importlib.util.spec_from_file_location("mk", os.path.join(HERE, "golden", "make_wide_k_digests.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    path = os.path.join(HERE, "golden", "wide_k_digests.txt")
    assert os.path.exists(path), "run tests/golden/make_wide_k_digests.py"
    rows = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        parts = line.split()
        rows[parts[0]] = ([int(v) for v in parts[1:10]], parts[10:])
    assert set(rows) == set(mk.CASES)
    for name, (vals, dg) in rows.items():
        assert tuple(vals) == mk.CASES[name]
        k, level = vals[6], vals[7]
        assert len(dg) == 2 * (level - k + 1)  # one digest per output limb of (c0, c1)
        assert all(len(d) == 16 and int(d, 16) >= 0 for d in dg)
