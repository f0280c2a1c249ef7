"""Autotuner: the tuned table round-trips through its JSON file, and the
factorization, solve and inversion agree with the oracle under the tuned
table and under every forced GEMM configuration (any configuration is
correct; only speed differs)."""
import json

import numpy as np
import pytest
import torch

import oracle
import paper_0901_1696_amd as rfp
import synth
from gpu_util import dev, dev_colmajor, host, host_colmajor, info_tensor, read_info

pytestmark = pytest.mark.gpu


def _check_all(h, n, transr, uplo, seed):
    A, B = synth.spd(n, nrhs=20, seed=seed)
    arf = oracle.trttf(transr, uplo, A)
    f, _ = oracle.pftrf(transr, uplo, n, arf.copy())
    x_want = oracle.pftrs(transr, uplo, n, f, B)
    inv_want, _ = oracle.pftri(transr, uplo, n, f)
    d = dev(arf)
    info = info_tensor()
    rfp.rfp_dpftrf(h, transr, uplo, n, d, info)
    assert read_info(info) == 0
    assert oracle.rel_fro(host(d), f) <= 1e-12 * n
    bd = dev_colmajor(B)
    rfp.rfp_dpftrs(h, transr, uplo, n, d, bd)
    assert oracle.rel_fro(host_colmajor(bd), x_want) <= 1e-12 * n
    rfp.rfp_dpftri(h, transr, uplo, n, d, info)
    assert read_info(info) == 0
    assert oracle.rel_fro(host(d), inv_want) <= 1e-12 * n


def test_autotune_roundtrip_and_parity(tmp_path):
    h = rfp.Handle(0)
    n = 700
    rfp.rfp_autotune(h, n, nrhs=20, precs=rfp.TUNE_FP64 | rfp.TUNE_FP32)
    count = rfp.rfp_tune_count(h)
    assert count > 0
    path = tmp_path / "tune.json"
    rfp.rfp_tune_save(h, str(path))
    doc = json.loads(path.read_text())  # valid JSON
    assert len(doc["gemm"]) + len(doc["solve"]) == count
    assert all(0 <= e["tile"] <= 3 for e in doc["gemm"])
    for t, u in oracle.LAYOUTS:
        _check_all(h, n, t, u, seed=5)
    rfp.rfp_tune_clear(h)
    assert rfp.rfp_tune_count(h) == 0
    rfp.rfp_tune_load(h, str(path))
    assert rfp.rfp_tune_count(h) == count
    path2 = tmp_path / "tune2.json"
    rfp.rfp_tune_save(h, str(path2))
    assert path2.read_text() == path.read_text()
    bad = tmp_path / "bad.json"
    bad.write_text('{"rfp_tune": 1,\n "gemm": [\n  {"key": 1, "dt": 0}\n ]\n}\n')
    with pytest.raises(rfp.RfpError):
        rfp.rfp_tune_load(h, str(bad))
    assert rfp.rfp_tune_count(h) == count  # a failed load keeps the table


@pytest.mark.parametrize("tile", [0, 1, 2, 3])
@pytest.mark.parametrize("split", [0, 1, 4])
def test_every_forced_configuration_is_correct(tile, split):
    h = rfp.Handle(0)
    rfp.rfp_tune_force(h, tile, split)
    for t, u, n in [("N", "L", 513), ("T", "U", 300), ("N", "U", 1001)]:
        _check_all(h, n, t, u, seed=n + tile)


def test_autotune_schedule(tmp_path):
    """The factorization schedule is tuned per size class: the tuned entry is
    saved and loaded with the table, factorizations of that class use it and
    stay correct, and a schedule set by the caller takes precedence."""
    h = rfp.Handle(0)
    n = 2300
    rfp.rfp_autotune(h, n, nrhs=0, precs=rfp.TUNE_SCHEDULE)
    assert rfp.rfp_tune_count(h) == 1
    path = tmp_path / "sched.json"
    rfp.rfp_tune_save(h, str(path))
    doc = json.loads(path.read_text())
    assert len(doc["sched"]) == 1
    e = doc["sched"][0]
    assert e["wide_panels_above"] in (3072, 6144, 12288, 2 ** 63 - 1)
    assert e["chunk_max"] in (1024, 1536, 2048) and e["leaf_lds_pad"] in (0, 24576)
    for t, u in [("N", "L"), ("T", "U")]:
        _check_all(h, n, t, u, seed=17)
    rfp.rfp_tune_clear(h)
    rfp.rfp_tune_load(h, str(path))
    assert rfp.rfp_tune_count(h) == 1
    rfp.rfp_set_schedule(h, dict(wide_panels_above=0))
    _check_all(h, n, "N", "U", seed=18)
    rfp.rfp_set_schedule(h, None)
