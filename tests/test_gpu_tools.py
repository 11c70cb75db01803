"""The launch-settings sweep on a small lattice (its output lines and best settings)."""
import pytest

from paper_1908_06742_amd import launch_sweep

pytestmark = pytest.mark.gpu


def test_launch_sweep_prints_every_setting_and_the_best(capsys):
    print("case: launch sweep 256^2 f32/f16", flush=True)
    launch_sweep.main(["--storage", "f32,f16", "--size", "256", "--tiles", "64,128", "--widths", "32",
                       "--caps", "0/0,1/2", "--pairs", "2"])
    out = capsys.readouterr().out.splitlines()
    rows = [l for l in out if "caps" in l]
    assert len(rows) == 2 * 2 * 2                     # storages x tiles x cap pairs
    assert all("even" in l and "odd" in l and "GB/s" in l for l in rows)
    best = [l for l in out if "best even" in l]
    assert len(best) == 2 and all("(64, 32" in l or "(128, 32" in l for l in best)
