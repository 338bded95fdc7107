"""Command-line front end: input parsing and output writing on the CPU; one
end-to-end run on the GPU against the oracle."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2412_04514_amd import cli

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_load_points_text_and_npy(tmp_path):
    t = tmp_path / "p.txt"
    t.write_text("# x y z\n0.1 0.2 0.3\n0.4,0.5,0.6  # comma separated\n\n0.7 0.8 0.9\n")
    P = cli.load_points(str(t))
    np.testing.assert_array_equal(P, [[0.1, 0.2, 0.3], [0.4, 0.5, 0.6], [0.7, 0.8, 0.9]])
    assert P.dtype == np.float64
    n = tmp_path / "p.npy"
    np.save(n, P.astype(np.float32))
    Q = cli.load_points(str(n))
    assert Q.dtype == np.float32 and Q.shape == (3, 3)


def test_load_points_rejects_bad_rows(tmp_path):
    t = tmp_path / "bad.txt"
    t.write_text("0.1 0.2\n")
    with pytest.raises(ValueError, match="expected 3 numbers"):
        cli.load_points(str(t))
    n = tmp_path / "bad.npy"
    np.save(n, np.zeros((4, 2)))
    with pytest.raises(ValueError, match="shape"):
        cli.load_points(str(n))


def test_write_result_text_and_npz(tmp_path):
    res = dict(row_ptr=np.array([0, 2, 3, 3]), col=np.array([1, 2, 0], np.int32), volume=np.ones(3), area=None)
    t = tmp_path / "o.txt"
    cli.write_result(str(t), res)
    assert t.read_text() == "1 2\n0\n\n"
    z = tmp_path / "o.npz"
    cli.write_result(str(z), res)
    with np.load(z) as d:
        assert set(d.files) == {"row_ptr", "col", "volume"}


def test_parser_defaults():
    a = cli.build_parser().parse_args(["p.npy", "-o", "o.npz"])
    assert a.box == [0.0, 0.0, 0.0, 1.0, 1.0, 1.0] and a.precision == "f64" and a.k0 == 32 and not a.faces


@pytest.mark.gpu
def test_cli_end_to_end(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    from paper_2412_04514_amd import gen
    P = gen.cluster(5000, seed=21, dtype=np.float64)
    src = tmp_path / "p.npy"
    np.save(src, P)
    out = tmp_path / "r.npz"
    r = subprocess.run([sys.executable, "-m", "paper_2412_04514_amd.cli", str(src), "-o", str(out), "--faces"],
                       cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["points"] == 5000
    orc = oracle.tessellate(P)
    with np.load(out) as d:
        assert np.array_equal(d["row_ptr"], orc["row_ptr"]) and np.array_equal(d["col"], orc["col"])
        np.testing.assert_allclose(d["volume"], orc["volume"], rtol=1e-12, atol=1e-14 / len(P))
        np.testing.assert_allclose(d["area"], orc["area"], rtol=1e-9, atol=1e-14)
        np.testing.assert_allclose(d["centroid"], orc["centroid"], rtol=0, atol=1e-12)
    txt = tmp_path / "r.txt"
    r = subprocess.run([sys.executable, "-m", "paper_2412_04514_amd.cli", str(src), "-o", str(txt)],
                       cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    rows = txt.read_text().splitlines()
    assert len(rows) == 5000
    assert [int(x) for x in rows[7].split()] == list(orc["col"][orc["row_ptr"][7]:orc["row_ptr"][8]])
