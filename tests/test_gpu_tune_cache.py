"""The sweep autotuner's results on disk (NLTE3D_TUNE_CACHE): written after tuning, read
by a new context (which then skips tuning and uses the stored shape), and a malformed file
is ignored."""
import json

import pytest

from paper_1701_01607_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nl():
    import torch
    assert torch.cuda.is_available()
    from paper_1701_01607_amd import nlte
    return nlte


def one_iteration(nl, atom, atm):
    import torch
    ctx = nl.Context(0, torch.cuda.current_stream().cuda_stream)
    M, A = ctx.atmos(atm), ctx.atom(atom)
    job = ctx.job(M, A, nl.SolveParams(method=nl.MALI, precision=nl.MIXED, nlev=1, max_iter=1, E_target=0.0,
                                       dirs_per_block=0))
    rc, r = job.run()
    job.close()
    M.close()
    A.close()
    ctx.close()
    return r.dirs_per_block


def test_tune_cache_round_trip(nl, tmp_path, monkeypatch):
    atom = synth.caii_like_atom(9)
    atm = synth.atmos_stratified(nx=96, ny=72, nz=5, dx=120 * synth.KM, seed=61)
    path = tmp_path / "tune.json"
    monkeypatch.setenv("NLTE3D_TUNE_CACHE", str(path))
    db = one_iteration(nl, atom, atm)
    entries = json.loads(path.read_text())
    assert db in (3, 6, 12)
    keys = [k for k in entries if k.endswith(":96x72x5:5:45")]
    assert len(keys) == 1 and entries[keys[0]] == db
    # a new context reads the file: force another shape there and it is used as is
    forced = 12 if db != 12 else 3
    entries[keys[0]] = forced
    entries["other-device|4:8x8x8:1:1"] = 6
    path.write_text(json.dumps(entries))
    assert one_iteration(nl, atom, atm) == forced
    assert json.loads(path.read_text())["other-device|4:8x8x8:1:1"] == 6
    # a malformed file is ignored: the shape is tuned again and the file rewritten
    path.write_text("{ not json")
    assert one_iteration(nl, atom, atm) in (3, 6, 12)
    assert len(json.loads(path.read_text())) == 1
