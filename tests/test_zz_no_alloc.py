"""The allocation-free training step (sel_mlp_train_step_noalloc) against the
one with a caller's work buffer (sel_mlp_train_step): two Adam steps in a
row, the second on fewer rows, give the same parameters, moments and loss
bit for bit (same kernels, same work layout); more rows than its fixed work
memory holds are refused."""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def _dp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def test_noalloc_train_step_matches_work_buffer_step():
    from paper_2509_19171_amd import inputs as I
    from paper_2509_19171_amd import sel

    assert torch.cuda.is_available()
    lib = sel.load()
    dev = torch.device("cuda:0")
    g = torch.Generator(device="cpu").manual_seed(11)
    rows = 6000
    X = torch.randn((rows, 6), generator=g).to(dev)
    y = torch.rand((rows,), generator=g).to(dev)
    blob = torch.tensor(I.closure_blob(3, mean=[0.0] * 6, std=[1.0] * 6), device=dev)
    st = torch.cuda.current_stream(dev)
    stream = ctypes.c_void_p(st.cuda_stream)
    sides = {}
    for name in ("work", "noalloc"):
        sides[name] = dict(p=blob.clone(), m=torch.zeros(8833, device=dev), v=torch.zeros(8833, device=dev))
    for t, n in ((1, 4096), (2, 1000)):
        idx = torch.randint(0, rows, (n,), generator=g, dtype=torch.int32).to(dev)
        losses = {}
        for name, sd in sides.items():
            loss = ctypes.c_double()
            if name == "work":
                work = torch.empty(int(lib.sel_mlp_work_floats(n)), dtype=torch.float32, device=dev)
                rc = lib.sel_mlp_train_step(_dp(sd["p"]), _dp(sd["m"]), _dp(sd["v"]), _dp(X), _dp(y), _dp(idx), n, t,
                                            1e-3, 0.9, 0.999, 1e-8, _dp(work), ctypes.byref(loss), stream)
            else:
                rc = lib.sel_mlp_train_step_noalloc(_dp(sd["p"]), _dp(sd["m"]), _dp(sd["v"]), _dp(X), _dp(y),
                                                    _dp(idx), n, t, 1e-3, 0.9, 0.999, 1e-8, ctypes.byref(loss),
                                                    stream)
            assert rc == 0, lib.sel_last_error().decode()
            losses[name] = loss.value
        torch.cuda.synchronize()
        say(f"step {t}, {n} rows: loss {losses['work']:.6e} / {losses['noalloc']:.6e}")
        assert losses["work"] == losses["noalloc"]
        for key in ("p", "m", "v"):
            assert torch.equal(sides["work"][key], sides["noalloc"][key]), key
    assert not torch.equal(sides["work"]["p"], blob)  # the steps changed the parameters
    # beyond the fixed work memory: refused before any launch
    idx = torch.zeros(4097, dtype=torch.int32, device=dev)
    sd = sides["noalloc"]
    rc = lib.sel_mlp_train_step_noalloc(_dp(sd["p"]), _dp(sd["m"]), _dp(sd["v"]), _dp(X), _dp(y), _dp(idx), 4097, 3,
                                        1e-3, 0.9, 0.999, 1e-8, None, stream)
    assert rc == sel.SEL_EINVAL and "4096" in lib.sel_last_error().decode()
