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
    # eight-wave form, one workgroup per bootstrap
    {"br_grid": 0, "latency_form_max": 1 << 30, "latency_waves": 8, "throughput_waves": 8, "ks_tile": 8},
    # eight-wave form with one LDS buffer, two per CU; key switch in tiles of 4
    {"br_grid": 0, "latency_form_max": 0, "latency_waves": 8, "throughput_waves": 8, "ks_tile": 4},
    # the same with a persistent grid of 7 workgroups that loop over the batch; tiles of 16
    {"br_grid": 7, "latency_form_max": 0, "latency_waves": 8, "throughput_waves": 8, "ks_tile": 16},
    # four-wave form, two per CU, and persistent
    {"br_grid": 0, "latency_form_max": 0, "latency_waves": 8, "throughput_waves": 4, "ks_tile": 8},
    {"br_grid": 7, "latency_form_max": 0, "latency_waves": 8, "throughput_waves": 4, "ks_tile": 16},
    # persistent eight-wave form
    {"br_grid": 5, "latency_form_max": 1 << 30, "latency_waves": 8, "throughput_waves": 8, "ks_tile": 4},
    # sixteen-wave form, and persistent
    {"br_grid": 0, "latency_form_max": 1 << 30, "latency_waves": 16, "throughput_waves": 8, "ks_tile": 8},
    {"br_grid": 3, "latency_form_max": 1 << 30, "latency_waves": 16, "throughput_waves": 8, "ks_tile": 8},
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


FORMS = {
    "sixteen_wave": {"br_grid": 0, "latency_form_max": 1 << 30, "latency_waves": 16, "throughput_waves": 8,
                     "ks_tile": 16},
    "eight_wave_two_per_cu": {"br_grid": 0, "latency_form_max": 0, "latency_waves": 8, "throughput_waves": 8,
                              "ks_tile": 4},
}


@pytest.mark.parametrize("form", sorted(FORMS))
def test_form_bit_exact(gpu, okeys, form):
    """The sixteen-wave form and the eight-wave form with two workgroups per
    CU on all 32 inputs of Table table_lutrelu and on an ASCII edit
    distance: every ciphertext bit-exact with the oracle."""
    from oracle import leuvenshtein as OL
    g = gpu
    L, torch = g.L, g.torch
    saved = L.lvs_context_get_tuning(g.ctx)
    try:
        L.lvs_context_set_tuning(g.ctx, FORMS[form])
        say(form, "table1 exhaustive")
        L.lvs_context_set_lut(g.ctx, L.LVS_LUT_USER, P.LUT_X_MINUS_4)
        cts = np.stack([L.lvs_lwe_encrypt(g.ck, x, 501, x) for x in range(32)])
        out = run_pbs(g, cts, L.LVS_LUT_USER)
        ref = okeys.pbs_batch(cts, T.test_polynomial(P.LUT_X_MINUS_4, 2048)[None, :], 0)
        for x in range(32):
            assert_same_ct(out[x], ref[x], f"x={x}")
        say(form, "kitten / sitting")
        a, b = b"kitten", b"sitting"
        A = L.lvs_encrypt_string(g.ck, a, L.LVS_ENC_ASCII7, 1001)
        B = L.lvs_encrypt_string(g.ck, b, L.LVS_ENC_ASCII7, 1002)
        d_h = torch.zeros(len(b) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
        L.lvs_edit_distance(g.ctx, L.to_device(A, g.dev), len(a), L.to_device(B, g.dev), len(b), L.LVS_ENC_ASCII7,
                            d_h)
        torch.cuda.synchronize()
    finally:
        L.lvs_context_set_tuning(g.ctx, saved)
    h = L.to_host(d_h).reshape(len(b), L.CT_WORDS)
    oh = OL.edit_distance(okeys, OL.encrypt_string(okeys, a, OL.ENC_ASCII7, 1001),
                          OL.encrypt_string(okeys, b, OL.ENC_ASCII7, 1002), OL.ENC_ASCII7)
    for j in range(len(b)):
        assert_same_ct(h[j], oh[j], f"h[m,{j + 1}]")
    assert L.lvs_decrypt_distance(g.ck, h, len(a)) == 3


def test_set_tuning_rejects_negative(gpu):
    L = gpu.L
    with pytest.raises(L.LvsError) as e:
        L.lvs_context_set_tuning(gpu.ctx, {"br_grid": -1, "latency_form_max": 0})
    assert e.value.code == -1
    with pytest.raises(L.LvsError) as e:
        L.lvs_context_set_tuning(gpu.ctx, {"br_grid": 0, "latency_form_max": 0, "latency_waves": 12})
    assert e.value.code == -1
    with pytest.raises(L.LvsError) as e:
        L.lvs_context_set_tuning(gpu.ctx, {"br_grid": 0, "latency_form_max": 0, "throughput_waves": 6})
    assert e.value.code == -1
    with pytest.raises(L.LvsError) as e:
        L.lvs_context_set_tuning(gpu.ctx, {"br_grid": 0, "latency_form_max": 0, "ks_tile": 5})
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
        assert {(cus, 1), (cus, 2), (cus, 3), (cus, 4), (cus, 5)} <= forms
        assert {r["grid"] for r in first["samples"] if r["form"] == 5} == {4, 8, 16}
        assert t["throughput_waves"] in (4, 8) and t["latency_waves"] in (8, 16) and t["ks_tile"] in (4, 8, 16)
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
