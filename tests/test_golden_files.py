"""The stored expected values are exactly what the oracle script writes (CPU only)."""
import importlib.util
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def test_golden_files_are_reproducible(oracle_native):
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "golden", "make_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    for name, text in mod.files().items():
        with open(os.path.join(HERE, "golden", name)) as f:
            assert f.read() == text, name
