"""Shared fixtures of the GPU parity tests: the HIP library's keys and device
context, and the oracle's keys drawn from the same seed."""
import sys

import numpy as np
import pytest

KEY_SEED = 1


def say(*args):
    """Name the case before each GPU step (flushed, so the output names it even if the process dies)."""
    print("[gpu-test]", *args, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="session")
def gpu():
    import torch
    from paper_2508_14568_amd import lvs as L
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    params = L.lvs_params_default()
    ck, sk = L.lvs_keygen(params, KEY_SEED)
    say("context create")
    ctx = L.lvs_context_create(sk, params, 0)
    torch.cuda.synchronize()

    class G:
        pass
    g = G()
    g.L, g.torch, g.params, g.ck, g.sk, g.ctx = L, torch, params, ck, sk, ctx
    g.dev = ctx.device
    return g


@pytest.fixture(scope="session")
def okeys():
    from oracle import tfhe as T
    return T.Keys(T.default_params(), seed=KEY_SEED)


@pytest.fixture(scope="session")
def okeys_kara():
    """The oracle's keys with Karatsuba's products in the blind rotation (the
    same words as the schoolbook sums, pinned by the oracle's tests; faster
    for the live runs of hundreds of bootstraps)."""
    from oracle import tfhe as T
    return T.Keys(T.default_params(), seed=KEY_SEED, karatsuba=True)


def oracle_threads():
    """Host threads for live oracle runs: the host cores, at most 16 (the CPU share of one GPU)."""
    import os
    return max(1, min(16, os.cpu_count() or 1))


def assert_same_ct(gpu_ct, oracle_ct, what=""):
    g = np.asarray(gpu_ct, dtype=np.uint64)
    o = np.asarray(oracle_ct, dtype=np.uint64)
    assert g.shape == o.shape, (what, g.shape, o.shape)
    diff = np.nonzero(g != o)
    assert diff[0].size == 0, f"{what}: {diff[0].size} words differ, first at {[int(x[0]) for x in diff]}"
