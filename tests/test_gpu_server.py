"""GPU tests of the projection server (lspca_server_*): each request's Z is
bitwise the same alone, in a mix of concurrent requests and as
lspca_transform, and within the projection bound of the FP64 oracle;
admission by arena memory, queue limits, time-outs and host requests."""
import numpy as np
import pytest

from oracle import lspca_oracle as O
from synth import lowrank_np, random_orthonormal_np, request_sizes, storage_to_f64
from tests.helpers import U32, U64, to_device

pytestmark = pytest.mark.gpu

CODE = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3}
SIZES = [1, 5, 127, 128, 129, 300, 1000, 2049, 4097]


def _pool(rows, n, dtype, seed=21):
    Xs = lowrank_np(rows, n, 16, "invsqrt", 0.05, seed, dtype)
    return Xs, storage_to_f64(Xs, dtype)


def _v(n, k, seed=3):
    import torch
    return torch.from_numpy(random_orthonormal_np(n, k, np.random.default_rng(seed))).cuda()


def _zdt(dtype):
    import torch
    return torch.float64 if dtype == "f64" else torch.float32


def _bound(X64, V, dtype):
    """Componentwise bound of Z = X V as lspca_transform computes it."""
    n = X64.shape[1]
    u = U64 if dtype == "f64" else U32
    aXV = np.abs(X64) @ np.abs(V)
    b = (n * u / (1 - n * u)) * aXV
    if dtype in ("bf16", "f16"):
        u16 = 2.0 ** -8 if dtype == "bf16" else 2.0 ** -11
        b = 2 * b + (1.01 * u16 ** 2 + U32 + 2.0 ** -24) * aXV
    elif dtype == "f32":
        b = b + U32 * aXV
    return b


def _slices(total, sizes, rng):
    out = []
    for r in sizes:
        r0 = int(rng.integers(0, total - r + 1))
        out.append((r0, r))
    return out


@pytest.mark.parametrize("dtype,n,k", [("bf16", 512, 256), ("bf16", 520, 64), ("f16", 384, 128),
                                       ("f32", 300, 40), ("f64", 200, 24),
                                       # the 4,097-row request's lspca_transform takes
                                       # the streamed FP32 kernel, the server the tiles
                                       ("f32", 256, 64)])
def test_alone_mix_and_transform_agree_bitwise(gpu_lib, dtype, n, k):
    import torch
    total = 6000
    Xs, X64 = _pool(total, n, dtype)
    X = to_device(Xs, dtype)
    V = _v(n, k)
    rng = np.random.default_rng(5)
    reqs = _slices(total, SIZES, rng)
    with gpu_lib.Server(V, CODE[dtype], max_inflight=64) as srv:
        # the server's streams do not wait on torch's: inputs and outputs
        # are made ready before submission
        alone = [torch.full((r, k), float("nan"), dtype=_zdt(dtype), device="cuda") for _, r in reqs]
        order = [i for _ in range(3) for i in rng.permutation(len(reqs))]
        outs = [(i, torch.full((reqs[i][1], k), float("nan"), dtype=_zdt(dtype), device="cuda"))
                for i in order]
        torch.cuda.synchronize()
        for (r0, r), Z in zip(reqs, alone):
            srv.wait(srv.submit(X[r0:r0 + r], Z))
        # the same requests, three times over in shuffled order, released at
        # once: they share launches
        srv.pause(True)
        tickets = [srv.submit(X[reqs[i][0]:reqs[i][0] + reqs[i][1]], Z) for i, Z in outs]
        srv.pause(False)
        for t in tickets:
            srv.wait(t)
        st = srv.stats()
    assert st["max_requests_per_launch"] > 1
    assert st["completed"] == st["submitted"] == len(reqs) + len(order)
    for i, Z in outs:
        assert torch.equal(Z, alone[i])
    Vn = V.cpu().numpy()
    Vq = Vn.astype(np.float32).astype(np.float64) if dtype == "f32" else Vn
    for (r0, r), Z in zip(reqs, alone):
        assert torch.equal(Z, gpu_lib.transform(X[r0:r0 + r], V))
        ref = O.transform(X64[r0:r0 + r], Vq)
        assert np.all(np.abs(Z.cpu().numpy().astype(np.float64) - ref) <= _bound(X64[r0:r0 + r], Vq, dtype))


def test_small_tile_class_gives_the_standard_bits(gpu_lib, monkeypatch):
    """A server whose requests all take the standard tiles (small class
    switched off) and the default one (requests of at most 4,096 rows in
    32 x 64 tiles) give the same bits, alone and with both classes in one
    launch."""
    import torch
    n, k, total = 4096, 256, 12000
    Xs, _ = _pool(total, n, "bf16", seed=14)
    X = to_device(Xs, "bf16")
    V = _v(n, k, seed=15)
    sizes = [1, 7, 64, 500, 4096, 4097, 9000, 3]
    rng = np.random.default_rng(6)
    reqs = _slices(total, sizes, rng)
    outs = {}
    for label, env in (("standard", "0"), ("default", None)):
        if env is None:
            monkeypatch.delenv("LSPCA_PROJ_SMALL_ROWS", raising=False)
        else:
            monkeypatch.setenv("LSPCA_PROJ_SMALL_ROWS", env)
        with gpu_lib.Server(V, CODE["bf16"], max_inflight=16) as srv:
            Zs = [torch.full((r, k), float("nan"), dtype=torch.float32, device="cuda") for _, r in reqs]
            Zm = [torch.full((r, k), float("nan"), dtype=torch.float32, device="cuda") for _, r in reqs]
            torch.cuda.synchronize()
            for (r0, r), Z in zip(reqs, Zs):                       # one at a time
                srv.wait(srv.submit(X[r0:r0 + r], Z))
            srv.pause(True)                                         # all in one launch
            tickets = [srv.submit(X[r0:r0 + r], Z) for (r0, r), Z in zip(reqs, Zm)]
            srv.pause(False)
            for t in tickets:
                srv.wait(t)
            assert srv.stats()["max_requests_per_launch"] == len(reqs)
        outs[label] = (Zs, Zm)
    monkeypatch.delenv("LSPCA_PROJ_SMALL_ROWS", raising=False)
    for i, (r0, r) in enumerate(reqs):
        ref = outs["standard"][0][i]
        assert torch.equal(outs["standard"][1][i], ref), r
        assert torch.equal(outs["default"][0][i], ref), r
        assert torch.equal(outs["default"][1][i], ref), r
        assert torch.equal(gpu_lib.transform(X[r0:r0 + r], V), ref), r


def test_overlapping_submissions_complete_correctly(gpu_lib):
    """Requests submitted while earlier ones run (no pause): log-uniform row
    counts as the serving workload, every result bitwise its lone value."""
    import torch
    n, k, total = 512, 256, 70000
    Xs, _ = _pool(total, n, "bf16", seed=4)
    X = to_device(Xs, "bf16")
    V = _v(n, k, seed=8)
    sizes = request_sizes(40, seed=12)
    rng = np.random.default_rng(2)
    reqs = _slices(total, sizes, rng)
    with gpu_lib.Server(V, CODE["bf16"], max_inflight=16) as srv:
        Zs = [torch.empty((r, k), dtype=torch.float32, device="cuda") for _, r in reqs]
        torch.cuda.synchronize()
        tickets = [srv.submit(X[r0:r0 + r], Z) for (r0, r), Z in zip(reqs, Zs)]
        lat = [srv.wait(t) for t in tickets]
        st = srv.stats()
    assert all(x >= 0 for x in lat)
    assert st["completed"] == len(reqs)
    for (r0, r), Z in zip(reqs, Zs):
        assert torch.equal(Z, gpu_lib.transform(X[r0:r0 + r], V))


def test_host_requests_are_admitted_by_arena_memory(gpu_lib):
    import torch
    n, k = 256, 64
    Xs, _ = _pool(4000, n, "bf16", seed=6)
    Xd = to_device(Xs, "bf16")
    V = _v(n, k, seed=9)
    rows = [700, 1500, 900, 1200, 333, 1000]
    per = max(((r * n * 2 + 255) // 256 * 256 + (r * k * 4 + 255) // 256 * 256) for r in rows)
    arena = 2 * per + 4096
    with gpu_lib.Server(V, CODE["bf16"], arena_bytes=arena, max_inflight=8) as srv:
        Xh = [Xd[:r].cpu().pin_memory() for r in rows]
        Zh = [torch.empty((r, k), dtype=torch.float32).pin_memory() for r in rows]
        torch.cuda.synchronize()
        tickets = [srv.submit(x, z) for x, z in zip(Xh, Zh)]
        for t in tickets:
            srv.wait(t)
        st = srv.stats()
        big = torch.empty((4000, n), dtype=torch.bfloat16).pin_memory()
        zbig = torch.empty((4000, k), dtype=torch.float32).pin_memory()
        with pytest.raises(gpu_lib.LspcaError) as e:
            srv.submit(big, zbig)
        assert e.value.name == "LSPCA_E2BIG"
        # device X with host Z: refused
        with pytest.raises(gpu_lib.LspcaError) as e:
            srv.submit(Xd[:10], zbig[:10])
        assert e.value.name == "LSPCA_EINVAL"
    assert 0 < st["arena_peak_bytes"] <= arena
    for r, z in zip(rows, Zh):
        assert torch.equal(z.cuda(), gpu_lib.transform(Xd[:r], V))


def test_queue_limit_timeout_and_tickets(gpu_lib):
    import torch
    n, k = 128, 32
    Xs, _ = _pool(500, n, "f32", seed=7)
    X = to_device(Xs, "f32")
    V = _v(n, k, seed=10)
    with gpu_lib.Server(V, CODE["f32"], max_inflight=1) as srv:
        srv.pause(True)
        Z = torch.empty((100, k), dtype=torch.float32, device="cuda")
        Zq = [torch.empty((50, k), dtype=torch.float32, device="cuda") for _ in range(20)]
        torch.cuda.synchronize()
        t0 = srv.submit(X[:100], Z)
        with pytest.raises(gpu_lib.LspcaError) as e:
            srv.wait(t0, timeout_us=2000)
        assert e.value.name == "LSPCA_ETIMEDOUT"
        accepted, refused = [t0], 0
        outs = [Z]
        for Zi in Zq:
            try:
                accepted.append(srv.submit(X[:50], Zi))
                outs.append(Zi)
            except gpu_lib.LspcaError as err:
                assert err.name == "LSPCA_EAGAIN"
                refused += 1
        # max_inflight = 1 admits one request; 16 may wait in the queue
        assert refused >= 1 and len(accepted) in (16, 17)
        srv.pause(False)
        for t in accepted:
            assert srv.wait(t) >= 0
        with pytest.raises(gpu_lib.LspcaError) as e:
            srv.wait(t0)
        assert e.value.name == "LSPCA_ENOTFOUND"
        # an empty request completes at once
        empty = torch.empty((0, n), dtype=torch.float32, device="cuda")
        assert srv.wait(srv.submit(empty, torch.empty((0, k), dtype=torch.float32, device="cuda")), 0) == 0
    ref = gpu_lib.transform(X[:100], V)
    assert torch.equal(outs[0], ref)
    for Zi in outs[1:]:
        assert torch.equal(Zi, ref[:50])


def test_destroy_finishes_submitted_requests(gpu_lib):
    import torch
    n, k = 256, 64
    Xs, _ = _pool(3000, n, "bf16", seed=8)
    X = to_device(Xs, "bf16")
    V = _v(n, k, seed=11)
    srv = gpu_lib.Server(V, CODE["bf16"], max_inflight=4)
    Zs = [(r, torch.full((r, k), float("nan"), dtype=torch.float32, device="cuda")) for r in (100, 2000, 3000, 17)]
    torch.cuda.synchronize()
    for r, Z in Zs:
        srv.submit(X[:r], Z)
    srv.close()
    torch.cuda.synchronize()
    for r, Z in Zs:
        assert torch.equal(Z, gpu_lib.transform(X[:r], V))
