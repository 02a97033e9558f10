"""The autotuner of the batched kernel: every configuration it may choose
gives the default configuration's results bit for bit, and a batch built with
tuning on equals the default batch (tolerance 0: integer observables)."""
import sys

import numpy as np
import pytest

from test_gpu_batch import _mixed_jobs, _same_obs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("L", [8, 24, 40, 64])
def test_tune_candidates_all_bit_exact(ea_gpu, L):
    r = ea_gpu.tune(L, force=True)
    _say(f"tune L={L}: chosen {r['chosen']}")
    for c in r["tried"]:
        _say(f"   {c}")
    assert len(r["tried"]) >= 2
    assert all(c["parity_ok"] for c in r["tried"])
    ch = r["chosen"]
    assert any((c["words_per_row"], c["threads"], c["select"]) ==
               (ch["words_per_row"], ch["threads"], ch["select"]) for c in r["tried"])
    assert ch["threads"] % 64 == 0 and 64 <= ch["threads"] <= 1024
    # a second call returns the cached choice without probing again
    again = ea_gpu.tune(L)
    assert again["tried"] == []
    assert (again["chosen"]["words_per_row"], again["chosen"]["threads"], again["chosen"]["select"]) == \
        (ch["words_per_row"], ch["threads"], ch["select"])


def test_batch_autotune_equals_default(ea_gpu):
    jobs = _mixed_jobs()
    d = ea_gpu.Batch(jobs)
    d.run()
    a = ea_gpu.Batch(jobs, autotune=True)
    a.run()
    for j, job in enumerate(jobs):
        for k in range(len(job.meas_t)):
            _same_obs(a.result(j, k), d.result(j, k), f"job {j} meas {k}")
        for r in (0, 1):
            assert np.array_equal(a.spins(j, r), d.spins(j, r)), (j, r)


def test_tune_rejects_bad_sizes(ea_gpu):
    for L in (0, 12, 72, 128):
        with pytest.raises(ea_gpu.EAError):
            ea_gpu.tune(L)


def test_tune_cache_file_roundtrip(ea_gpu, tmp_path):
    """EA_TUNE_CACHE: a first process tunes and appends its choices, a second
    process reads them back without probing."""
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune_cache.txt"
    env = dict(os.environ, EA_TUNE_CACHE=str(cache))
    code = ("import paper_1411_5512_amd as ea; r = ea.tune(16); p = ea.tune_plain(24); "
            "c = r['chosen']; print(c['words_per_row'], c['threads'], c['select'], len(r['tried']), "
            "p['words_per_row'], len(p['tried']))")

    def run():
        out = subprocess.run([sys.executable, "-c", code], env=env, cwd=root, capture_output=True, text=True,
                             timeout=300)
        assert out.returncode == 0, out.stderr[-2000:]
        return out.stdout.split()

    first = run()
    assert int(first[3]) >= 2 and int(first[5]) >= 2  # probed
    lines = cache.read_text().splitlines()
    assert any(" batch 16 " in ln for ln in lines) and any(" plain 24 " in ln for ln in lines)
    second = run()
    assert second[3] == "0" and second[5] == "0"  # read from the file
    assert second[:3] == first[:3] and second[4] == first[4]
