"""lam_decode_forward_noalloc: the inference decode without a workspace (its
dictionary scratch is the library's static per-GPU array) gives exactly what
lam_decode_forward gives, call after call, including a smaller second call,
under HIP-graph capture, and refuses a dictionary beyond the scratch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from tests.gpu_helpers import say, to_np  # noqa: E402

pytestmark = pytest.mark.gpu


def _inputs(seed, n, d, M, D):
    rng = np.random.default_rng(seed)
    f = lambda *s: torch.as_tensor(rng.standard_normal(s).astype(np.float32), device="cuda")
    return f(n, d), f(M, d), f(M, D)


def _reference(prec, Q, K, V):
    from paper_2602_12314_amd import ops
    n, d = Q.shape
    M, D = V.shape
    F = ops.Decoder(prec, n, d, M, D).forward(Q, K, V)
    torch.cuda.synchronize()
    return to_np(F)


def _noalloc(prec, Q, K, V):
    from paper_2602_12314_amd import _lib
    F = torch.full((Q.shape[0], V.shape[1]), float("nan"), device="cuda")
    _lib.decode_forward_noalloc(prec, Q, K, V, F)
    torch.cuda.synchronize()
    return to_np(F)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_noalloc_equals_workspace_decode_twice(prec):
    # the second call is smaller in every dimension (fewer pixels, atoms and
    # feature columns) and must not see the first call's scratch contents
    big = (3000, 32, 960 if prec == "fp32" else 1536, 1024)
    small = (517, 16, 100, 256)
    for k, (n, d, M, D) in enumerate((big, small)):
        say(f"[noalloc] {prec} call {k + 1}: n={n} d={d} M={M} D={D}")
        Q, K, V = _inputs(10 + k, n, d, M, D)
        got = _noalloc(prec, Q, K, V)
        ref = _reference(prec, Q, K, V)
        assert np.array_equal(got, ref), (prec, k)


def test_noalloc_under_graph_capture():
    from paper_2602_12314_amd import _lib
    n, d, M, D = 2048, 16, 256, 512
    say(f"[noalloc] bf16 under HIP-graph capture n={n} d={d} M={M} D={D}")
    Q, K, V = _inputs(3, n, d, M, D)
    ref = _reference("bf16", Q, K, V)
    F = torch.zeros((n, D), device="cuda")
    _lib.decode_forward_noalloc("bf16", Q, K, V, F)  # first use on the context, outside capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            _lib.decode_forward_noalloc("bf16", Q, K, V, F)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        F.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(to_np(F), ref), rep
        # other work on the same scratch between replays (a different dictionary)
        Q2, K2, V2 = _inputs(20 + rep, 300, 32, 64, 128)
        _noalloc("fp32", Q2, K2, V2)


def test_noalloc_refuses_dictionary_beyond_scratch():
    from paper_2602_12314_amd import _lib
    Q, K, V = _inputs(4, 64, 32, 2048, 1024)  # BF16: 2048 x (32 + 2048 + 32) x 2 bytes > 8 MiB
    F = torch.empty((64, 1024), device="cuda")
    with pytest.raises(_lib.LamError) as e:
        _lib.decode_forward_noalloc("bf16", Q, K, V, F)
    assert e.value.status == _lib.LAM_ERR_UNSUPPORTED
    Qf, Kf, Vf = _inputs(5, 64, 32, 1024, 1024)  # FP32 at M = D = 1024 needs 16.9 MB
    with pytest.raises(_lib.LamError) as e:
        _lib.decode_forward_noalloc("fp32", Qf, Kf, Vf, F)
    assert e.value.status == _lib.LAM_ERR_UNSUPPORTED
