"""Launch shapes of the blind rotation (lvs_context_set_tuning, lvs_autotune):
every shape gives bit-identical bootstraps, equal to the oracle's; the
autotuner installs a valid shape and its JSON cache round-trips."""
import json

import numpy as np
import pytest

from gpu_common import assert_same_ct, gpu, okeys, say  # noqa: F401
from oracle import plaintext as P
from oracle import tfhe as T

pytestmark = pytest.mark.gpu

SHAPES = [
    {"br_grid": 0, "latency_form_max": 1 << 30},   # eight-wave form, one workgroup per bootstrap
    {"br_grid": 0, "latency_form_max": 0},         # four-wave form, two per CU
    {"br_grid": 7, "latency_form_max": 0},         # persistent four-wave form, 7 workgroups loop
    {"br_grid": 5, "latency_form_max": 1 << 30},   # persistent eight-wave form
]


def run_pbs(g, cts, lut_id):
    d_in = g.L.to_device(cts, g.dev)
    d_out = g.torch.zeros_like(d_in)
    g.L.lvs_pbs_batch(g.ctx, d_in, len(cts), d_out, lut_id=lut_id)
    g.torch.cuda.synchronize()
    return g.L.to_host(d_out).reshape(len(cts), g.L.CT_WORDS)


def test_every_shape_bit_identical(gpu, okeys):
    g = gpu
    L = g.L
    saved = L.lvs_context_get_tuning(g.ctx)
    rng = np.random.default_rng(17)
    mus = rng.integers(0, 32, size=23)
    cts = np.stack([L.lvs_lwe_encrypt(g.ck, int(mu), 900, k) for k, mu in enumerate(mus)])
    outs = []
    try:
        for sh in SHAPES:
            say("shape", sh)
            L.lvs_context_set_tuning(g.ctx, sh)
            assert L.lvs_context_get_tuning(g.ctx) == sh
            outs.append(run_pbs(g, cts, L.LVS_LUT_MIN))
    finally:
        L.lvs_context_set_tuning(g.ctx, saved)
    for o in outs[1:]:
        assert (o == outs[0]).all()
    ref = okeys.pbs_batch(cts[:3], T.test_polynomial(P.lut_min_negated(), 2048), 0)
    for b in range(3):
        assert_same_ct(outs[0][b], ref[b], f"b={b}")


def test_set_tuning_rejects_negative(gpu):
    L = gpu.L
    with pytest.raises(L.LvsError) as e:
        L.lvs_context_set_tuning(gpu.ctx, {"br_grid": -1, "latency_form_max": 0})
    assert e.value.code == -1


def test_autotune_and_cache(gpu, tmp_path):
    g = gpu
    L = g.L
    saved = L.lvs_context_get_tuning(g.ctx)
    say("autotune")
    try:
        path = str(tmp_path / "tuning.json")
        first = L.autotune(g.ctx, max_batch=512, cache=path)
        assert not first["cached"]
        cus = g.torch.cuda.get_device_properties(g.dev).multi_processor_count
        t = first["tuning"]
        assert t["br_grid"] in (0, 2 * cus)
        assert 0 <= t["latency_form_max"] <= 512 or t["latency_form_max"] == 2 ** 31 - 1
        forms = {(r["batch"], r["form"]) for r in first["samples"]}
        assert (cus, 1) in forms and (cus, 2) in forms
        assert all(r["ms"] > 0 for r in first["samples"])
        assert L.lvs_context_get_tuning(g.ctx) == t
        with open(path) as f:
            assert len(json.load(f)) == 1
        L.lvs_context_set_tuning(g.ctx, saved)
        second = L.autotune(g.ctx, max_batch=512, cache=path)
        assert second["cached"] and second["tuning"] == t
        assert L.lvs_context_get_tuning(g.ctx) == t
    finally:
        L.lvs_context_set_tuning(g.ctx, saved)
