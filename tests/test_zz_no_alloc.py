"""lbm_totals_noalloc, the entry point for callers that cannot allocate:
FP64 conservation totals of populations held in caller device memory, with
the partial sums in the library's fixed device array, against lbm_totals
of a context holding the same populations. Two calls in a row, the second
on a smaller box (the fixed array keeps the first call's contents)."""
import numpy as np
import pytest

from paper_1909_08406_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    from paper_1909_08406_amd import lbm
    return lbm


def say(*a):
    print(*a, flush=True)


def _stored(L, f, storage, shift_exp, rho0=1.0):
    """The stored values of decoded FP64 populations f [41, N]: f itself, or
    (f - w rho0) 2^k_q with k_q = round(-log2 w_q) + shift_exp, checked to
    decode back to f exactly."""
    _, w, _ = L.lattice()
    if storage in ("f64", "f32"):
        return f
    k = np.round(-np.log2(w)) + shift_exp if storage != "f32s" else np.zeros(41)
    h = (f - w[:, None] * rho0) * np.exp2(k)[:, None]
    assert np.array_equal(w[:, None] * rho0 + h * np.exp2(-k)[:, None], f)
    return h


def _device(torch, h, storage):
    dt = {"f64": torch.float64, "f32": torch.float32, "f32s": torch.float32, "f16s": torch.float16,
          "bf16s": torch.bfloat16}[storage]
    d = torch.tensor(h, dtype=torch.float64, device="cuda").to(dt).contiguous()
    # the conversion is exact: the values are the held ones
    assert np.array_equal(d.to(torch.float64).cpu().numpy(), h)
    return d


@pytest.mark.parametrize("storage,sr", [("f64", False), ("f32", False), ("f16s", True), ("bf16s", False),
                                        ("f32s", False)])
def test_totals_noalloc_matches_lbm_totals(L, storage, sr):
    import torch
    _, _, th = L.lattice()
    stream = torch.cuda.current_stream()
    for dims, seed in (((24, 12, 10), 3), ((7, 5, 3), 4)):  # the second call on a smaller box
        F = wl.random_state(*dims, seed=seed, amp_u=0.05, amp_rho=1e-2, amp_theta=2e-2)
        ctx = L.init([(*dims, 0.6)], *F.absolute(th), storage=storage, stochastic=sr)
        ctx.step(25)
        ref = ctx.totals()[0]
        f = ctx.get_populations().reshape(41, -1)
        kamp = ctx.info()["shift_exp"]
        ctx.free()
        N = f.shape[1]
        d = _device(torch, _stored(L, f, storage, kamp), storage)
        out = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
        L.totals_noalloc(d.data_ptr(), storage, dims, N, 1.0, kamp, stream, out.data_ptr())
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        say("noalloc %s %s: %s vs lbm_totals %s" % (storage, dims, got, ref))
        assert np.array_equal(got, ref), (storage, dims, got - ref)


def test_totals_noalloc_rejects_bad_sizes(L):
    import torch
    d = torch.zeros(41 * 16, dtype=torch.float64, device="cuda")
    out = torch.zeros(5, dtype=torch.float64, device="cuda")
    # q-stride shorter than the box, a box beyond 2^32 nodes, unknown storage
    for args in (("f64", (2, 2, 2), 15), ("f64", (2048, 2048, 1024), 1 << 33), (9, (2, 2, 2), 16)):
        with pytest.raises(L.LbmError) as e:
            L.totals_noalloc(d.data_ptr(), args[0], args[1], args[2], 1.0, 0, None, out.data_ptr())
        assert e.value.code == L.E_ARG
