"""bench.py on the command line (host only): more than one GPU is refused
with a message and a non-zero status before anything touches a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_lattice_option_is_checked():
    """--q takes the two 3D lattices only; a bad value is an argument error
    (status 2) before any device work."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--q", "9"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and "--q" in r.stderr and r.stdout == ""


def test_stored_counters_are_keyed_on_the_workload():
    """The HBM counters stored beside the traces name the workload they were
    taken on, in the form bench.py matches against its own arguments."""
    import json

    with open(os.path.join(ROOT, "profiles", "tgv3d_n7_q27_fp32dev_hbm_counters.json")) as fh:
        cnt = json.load(fh)
    assert cnt["workload"] == "tgv3d 16^3 N=7 D3Q27" and cnt["precision"] == "fp32dev"
