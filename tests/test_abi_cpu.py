"""The C ABI library without a GPU: it loads, exports every symbol the header
declares, sizes workspaces, and rejects invalid arguments before any HIP
call (no compute runs here)."""
import ctypes as C

import pytest

import paper_2406_05061_amd as P
from paper_2406_05061_amd import progot as B


def test_library_exports_header_symbols():
    syms = P.header_symbols()
    assert {"pot_prepare_clouds", "pot_sinkhorn_solve", "pot_entropic_map", "pot_progot_solve",
            "pot_progot_map", "pot_marginal_check", "pot_workspace_bytes"} <= set(syms)
    lib = P.lib()
    for s in syms:
        assert hasattr(lib, s), s
    assert P.version().count(".") == 2


def test_status_strings():
    assert P.status_string(0) == "ok"
    for code in (1, -1, -2, -3, -4):
        assert P.status_string(code) not in ("ok", "unknown status")
    assert P.status_string(99) == "unknown status"


def test_workspace_bytes():
    assert P.workspace_bytes(0, 10, 4) == 0
    assert P.workspace_bytes(10, 0, 4) == 0
    assert P.workspace_bytes(10, 10, 0) == 0
    assert P.workspace_bytes(10, 10, 257) == 0
    w32 = P.workspace_bytes(1000, 700, 64, "fp32")
    w16 = P.workspace_bytes(1000, 700, 64, "bf16")
    assert w32 > 1000 * 64 * 4 and w16 > w32
    assert w32 % 256 == 0
    # grows with every size
    assert P.workspace_bytes(2000, 700, 64) > w32
    assert P.workspace_bytes(1000, 1400, 64) > w32


def _fake_clouds(n=8, m=8, d=4, ws_bytes=None):
    c = B.pot_clouds()
    c.n, c.m, c.d, c.precision = n, m, d, 0
    c.X = c.Y = c.xk = 0x1000
    c.ws = 0x2000
    c.ws_bytes = P.workspace_bytes(n, m, d) if ws_bytes is None else ws_bytes
    return c


def test_prepare_rejects_invalid_before_launch():
    lib = P.lib()
    c = B.pot_clouds()
    nb = P.workspace_bytes(8, 8, 4)
    inv = B.POT_ERR_INVALID
    # null inputs / workspace, bad sizes, bad precision
    assert lib.pot_prepare_clouds(C.byref(c), None, 8, 0x1000, 8, 4, None, None, 0, 0x2000, nb, None) == inv
    assert lib.pot_prepare_clouds(C.byref(c), 0x1000, 8, None, 8, 4, None, None, 0, 0x2000, nb, None) == inv
    assert lib.pot_prepare_clouds(C.byref(c), 0x1000, 8, 0x1000, 8, 4, None, None, 0, None, nb, None) == inv
    assert lib.pot_prepare_clouds(C.byref(c), 0x1000, 0, 0x1000, 8, 4, None, None, 0, 0x2000, nb, None) == inv
    assert lib.pot_prepare_clouds(C.byref(c), 0x1000, 8, 0x1000, 8, 300, None, None, 0, 0x2000, nb, None) == inv
    assert lib.pot_prepare_clouds(C.byref(c), 0x1000, 8, 0x1000, 8, 4, None, None, 7, 0x2000, nb, None) == inv
    assert lib.pot_prepare_clouds(None, 0x1000, 8, 0x1000, 8, 4, None, None, 0, 0x2000, nb, None) == inv
    # workspace too small
    assert lib.pot_prepare_clouds(C.byref(c), 0x1000, 8, 0x1000, 8, 4, None, None, 0, 0x2000, nb - 1,
                                  None) == B.POT_ERR_NOMEM


def test_solvers_reject_invalid_before_launch():
    lib = P.lib()
    inv = B.POT_ERR_INVALID
    c = _fake_clouds()
    info = B.pot_sinkhorn_info()
    f = g = 0x3000
    # eps <= 0, nan, tau < 0, max_iter < 1, null outputs, undersized workspace
    assert lib.pot_sinkhorn_solve(C.byref(c), 0.0, 1e-3, 10, None, None, f, g, C.byref(info), None) == inv
    assert lib.pot_sinkhorn_solve(C.byref(c), float("nan"), 1e-3, 10, None, None, f, g, None, None) == inv
    assert lib.pot_sinkhorn_solve(C.byref(c), 1.0, -1.0, 10, None, None, f, g, None, None) == inv
    assert lib.pot_sinkhorn_solve(C.byref(c), 1.0, 1e-3, 0, None, None, f, g, None, None) == inv
    assert lib.pot_sinkhorn_solve(C.byref(c), 1.0, 1e-3, 10, None, None, None, g, None, None) == inv
    assert lib.pot_sinkhorn_solve(None, 1.0, 1e-3, 10, None, None, f, g, None, None) == inv
    small = _fake_clouds(ws_bytes=16)
    assert lib.pot_sinkhorn_solve(C.byref(small), 1.0, 1e-3, 10, None, None, f, g, None, None) == inv
    # entropic map: alpha out of [0, 1], eps <= 0, null query with nq > 0
    assert lib.pot_entropic_map(C.byref(c), g, 1.0, f, 4, 1.5, f, None) == inv
    assert lib.pot_entropic_map(C.byref(c), g, -1.0, f, 4, 0.5, f, None) == inv
    assert lib.pot_entropic_map(C.byref(c), g, 1.0, None, 4, 0.5, f, None) == inv
    assert lib.pot_entropic_map(C.byref(c), g, 1.0, None, 0, 0.5, None, None) == B.POT_OK
    # progot: K out of range, bad schedules
    p = B.pot_progot_params()
    p.K, p.alpha_sched, p.eps_mode, p.theta = 0, 0, 0, 1.0
    p.tau_first = p.tau_last = 1e-3
    p.max_iter = 100
    pi = B.pot_progot_info()
    assert lib.pot_progot_solve(C.byref(c), C.byref(p), f, g, None, C.byref(pi), None) == inv
    p.K = 65
    assert lib.pot_progot_solve(C.byref(c), C.byref(p), f, g, None, C.byref(pi), None) == inv
    p.K, p.theta = 4, 0.0
    assert lib.pot_progot_solve(C.byref(c), C.byref(p), f, g, None, C.byref(pi), None) == inv
    p.theta, p.eps_mode = 1.0, 1  # explicit schedule without values
    assert lib.pot_progot_solve(C.byref(c), C.byref(p), f, g, None, C.byref(pi), None) == inv
    p.eps_mode, p.alpha_sched = 0, 3
    assert lib.pot_progot_solve(C.byref(c), C.byref(p), f, g, None, C.byref(pi), None) == inv
    eps = (C.c_float * 2)(1.0, -1.0)
    al = (C.c_float * 2)(0.5, 1.0)
    assert lib.pot_progot_map(C.byref(c), 2, g, eps, al, f, 4, f, None) == inv
    out = (C.c_double * 3)()
    assert lib.pot_marginal_check(C.byref(c), f, g, 0.0, out, None) == inv
    assert lib.pot_marginal_check(C.byref(c), None, g, 1.0, out, None) == inv


def test_binding_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    X = torch.zeros(4, 2)
    with pytest.raises(TypeError):
        P.prepare_clouds(X, X)


def test_server_rejects_invalid_before_device_work():
    lib = P.lib()
    inv = B.POT_ERR_INVALID
    h = C.c_void_p()
    assert P.Server.request_bytes(0, 10, 4) == 0
    assert P.Server.request_bytes(100, 100, 64) >= P.workspace_bytes(100, 100, 64)
    assert lib.pot_server_arena_overhead(0) == 0
    assert lib.pot_server_arena_overhead(4) > 0
    assert lib.pot_server_create(None, 0x1000, 1 << 30, 4, None) == inv
    assert lib.pot_server_create(C.byref(h), None, 1 << 30, 4, None) == inv
    assert lib.pot_server_create(C.byref(h), 0x1000, 1 << 30, 0, None) == inv
    assert lib.pot_server_create(C.byref(h), 0x1000, 1 << 30, 100000, None) == inv
    assert lib.pot_server_create(C.byref(h), 0x1000, 16, 4, None) == B.POT_ERR_NOMEM
    assert lib.pot_server_step(None, None, None) == inv
    assert lib.pot_server_poll(None, 1, None) == inv
    assert lib.pot_server_destroy(None) == inv
    rid = C.c_int64()
    p = B.pot_progot_params()
    assert lib.pot_server_submit(None, 0x1000, 8, 0x1000, 8, 4, C.byref(p), 0x1, 0x1, None,
                                 C.byref(rid)) == inv


def test_eps_schedule_rejects_invalid_before_launch():
    lib = P.lib()
    inv = B.POT_ERR_INVALID
    assert lib.pot_eps_schedule_bytes(0, 10, 4, 7) == 0
    assert lib.pot_eps_schedule_bytes(10, 0, 4, 7) == 0
    assert lib.pot_eps_schedule_bytes(10, 10, 4, 0) == 0
    assert lib.pot_eps_schedule_bytes(10, 10, 4, 65) == 0
    nb = lib.pot_eps_schedule_bytes(100, 50, 4, 7)
    assert nb > P.workspace_bytes(100, 100, 4) and nb % 256 == 0
    assert lib.pot_eps_schedule_bytes(100, 50, 4, 8) > nb
    c = _fake_clouds(8, 8, 4)
    grid = (C.c_double * 3)(0.5, 1.0, 2.0)
    bad = (C.c_double * 3)(0.5, -1.0, 2.0)
    eps = (C.c_double * 4)()
    wsb = lib.pot_eps_schedule_bytes(8, 5, 4, 3)
    args = dict(Yt=0x4000, mt=5, K=4, sched=0, grid=grid, G=3, beta0=5.0, tau=1e-3, it=100,
                eps=eps, ws=0x2000, wsb=wsb)

    def call(**kw):
        a = dict(args, **kw)
        return lib.pot_eps_schedule(C.byref(c), a["Yt"], a["mt"], a["K"], a["sched"], a["grid"], a["G"],
                                    a["beta0"], a["tau"], a["it"], a["eps"], None, None, a["ws"],
                                    a["wsb"], None)
    assert call(Yt=None) == inv
    assert call(mt=0) == inv
    assert call(K=0) == inv and call(K=65) == inv
    assert call(sched=3) == inv
    assert call(grid=bad) == inv
    assert call(G=0) == inv
    assert call(beta0=0.0) == inv and call(tau=0.0) == inv and call(it=0) == inv
    assert call(eps=None) == inv
    assert call(ws=None) == inv
    assert call(wsb=wsb - 1) == B.POT_ERR_NOMEM
    assert lib.pot_eps_schedule(None, 0x4000, 5, 4, 0, grid, 3, 5.0, 1e-3, 100, eps, None, None,
                                0x2000, wsb, None) == inv


def test_metrics_reject_invalid_before_launch():
    lib = P.lib()
    inv = B.POT_ERR_INVALID
    c = _fake_clouds(8, 6, 4)
    out = (C.c_double * 6)()
    assert lib.pot_coupling_metrics(C.byref(c), 0x3000, 0x3000, 0.0, out, None) == inv
    assert lib.pot_coupling_metrics(C.byref(c), None, 0x3000, 1.0, out, None) == inv
    assert lib.pot_coupling_metrics(C.byref(c), 0x3000, 0x3000, 1.0, None, None) == inv
    assert lib.pot_diag_metrics(C.byref(c), 0x3000, 0x3000, 1.0, out, None) == inv   # n != m
    assert lib.pot_sinkhorn_divergence_bytes(0, 5, 4) == 0
    nb = lib.pot_sinkhorn_divergence_bytes(100, 50, 4)
    assert nb >= P.workspace_bytes(100, 100, 4)
    o5 = (C.c_double * 5)()
    assert lib.pot_sinkhorn_divergence(0x1000, 100, 0x1000, 50, 4, None, None, -1.0, 1e-3, 10, o5,
                                       0x2000, nb, None) == inv
    assert lib.pot_sinkhorn_divergence(0x1000, 100, 0x1000, 50, 4, None, None, 0.0, 0.0, 10, o5,
                                       0x2000, nb, None) == inv
    assert lib.pot_sinkhorn_divergence(None, 100, 0x1000, 50, 4, None, None, 0.0, 1e-3, 10, o5,
                                       0x2000, nb, None) == inv
    assert lib.pot_sinkhorn_divergence(0x1000, 100, 0x1000, 50, 4, None, None, 0.0, 1e-3, 10, o5,
                                       0x2000, nb - 1, None) == B.POT_ERR_NOMEM


def test_pcost_workspace_and_prepare_reject_invalid():
    lib = P.lib()
    inv = B.POT_ERR_INVALID
    AUTO, FLY, KEEP = 0, 1, 2
    for p in (0.0, 0.5, 1.0, float("nan"), float("inf"), 17.0):
        assert lib.pot_workspace_bytes_pcost(100, 80, 8, p, AUTO) == 0, p
    assert lib.pot_workspace_bytes_pcost(0, 80, 8, 1.5, AUTO) == 0
    assert lib.pot_workspace_bytes_pcost(100, 80, 257, 1.5, AUTO) == 0
    assert lib.pot_workspace_bytes_pcost(100, 80, 8, 1.5, 3) == 0          # unknown flags
    # a kept matrix is limited to 2^36 entries; on the fly only the grid limits n m
    assert lib.pot_workspace_bytes_pcost(1 << 20, 1 << 20, 8, 1.5, KEEP) == 0
    big = lib.pot_workspace_bytes_pcost(1 << 20, 1 << 20, 8, 1.5, AUTO)
    assert 0 < big < (1 << 36)                                              # > 16 GiB: not kept
    assert lib.pot_workspace_bytes_pcost(1 << 22, 1 << 22, 8, 1.5, FLY) == 0  # grid limit
    nb = lib.pot_workspace_bytes_pcost(100, 80, 8, 1.5, AUTO)
    # the kept cost matrix (n x m rounded up to 4) is part of the workspace
    assert nb >= P.workspace_bytes(100, 80, 8) + 100 * 80 * 4 and nb % 256 == 0
    assert lib.pot_workspace_bytes_pcost(100, 80, 8, 1.5, KEEP) == nb
    assert lib.pot_workspace_bytes_pcost(100, 80, 8, 1.5, FLY) <= nb - 100 * 80 * 4
    assert lib.pot_workspace_bytes_pcost(100, 81, 8, 2.5, AUTO) > nb
    assert P.workspace_bytes(100, 80, 8, "bf16", cost_p=1.5) == 0
    c = B.pot_clouds()
    call = lambda **kw: lib.pot_prepare_clouds_pcost(
        C.byref(c), kw.get("X", 0x1000), kw.get("n", 100), kw.get("Y", 0x1000), kw.get("m", 80),
        kw.get("d", 8), None, None, kw.get("p", 1.5), kw.get("flags", AUTO), kw.get("ws", 0x2000),
        kw.get("wsb", nb), None)
    assert call(X=None) == inv and call(Y=None) == inv and call(ws=None) == inv
    assert call(p=1.0) == inv and call(p=0.0) == inv and call(n=0) == inv and call(d=300) == inv
    assert call(flags=7) == inv
    assert call(wsb=nb - 1) == B.POT_ERR_NOMEM


def test_pcost_clouds_validated():
    """A general-cost pot_clouds needs FP32, its cost matrix and its stride;
    the scheduler asks for its own workspace size."""
    lib = P.lib()
    inv = B.POT_ERR_INVALID
    c = _fake_clouds(8, 8, 4)
    c.cost_p = 1.5
    c.ws_bytes = lib.pot_workspace_bytes_pcost(8, 8, 4, 1.5, 2)
    info = B.pot_sinkhorn_info()
    # a stride without a matrix, or a matrix with the wrong stride
    c.cmat, c.ldc = 0, 8
    assert lib.pot_sinkhorn_solve(C.byref(c), 1.0, 1e-3, 10, None, None, 0x3000, 0x3000,
                                  C.byref(info), None) == inv
    c.cmat, c.ldc = 0x5000, 7
    assert lib.pot_sinkhorn_solve(C.byref(c), 1.0, 1e-3, 10, None, None, 0x3000, 0x3000,
                                  C.byref(info), None) == inv
    c.ldc = 8
    c.ws_bytes = lib.pot_workspace_bytes_pcost(8, 8, 4, 1.5, 1)   # too small for the matrix
    assert lib.pot_sinkhorn_solve(C.byref(c), 1.0, 1e-3, 10, None, None, 0x3000, 0x3000,
                                  C.byref(info), None) == inv
    c.ws_bytes = lib.pot_workspace_bytes_pcost(8, 8, 4, 1.5, 2)
    c.precision = 1
    assert lib.pot_entropic_map(C.byref(c), 0x3000, 1.0, 0x3000, 4, 1.0, 0x3000, None) == inv
    c.precision = 0
    # Alg. 4 on general-cost clouds takes the general-cost workspace
    grid = (C.c_double * 3)(0.5, 1.0, 2.0)
    eps = (C.c_double * 4)()
    wsb = lib.pot_eps_schedule_pcost_bytes(8, 5, 4, 3, 1.5)
    assert wsb >= lib.pot_workspace_bytes_pcost(8, 8, 4, 1.5, 0) and wsb % 256 == 0
    assert lib.pot_eps_schedule_pcost_bytes(8, 5, 4, 3, 1.0) == 0
    assert lib.pot_eps_schedule(C.byref(c), 0x4000, 5, 4, 0, grid, 3, 5.0, 1e-3, 100, eps, None,
                                None, 0x2000, wsb - 1, None) == B.POT_ERR_NOMEM


def test_pcost_divergence_rejects_invalid():
    lib = P.lib()
    inv = B.POT_ERR_INVALID
    assert lib.pot_sinkhorn_divergence_pcost_bytes(100, 80, 8, 1.0) == 0
    assert lib.pot_sinkhorn_divergence_pcost_bytes(0, 80, 8, 1.5) == 0
    nb = lib.pot_sinkhorn_divergence_pcost_bytes(100, 80, 8, 1.5)
    assert nb >= lib.pot_workspace_bytes_pcost(100, 100, 8, 1.5, 0) and nb % 256 == 0
    out = (C.c_double * 5)()
    call = lambda **kw: lib.pot_sinkhorn_divergence_pcost(
        kw.get("X", 0x1000), 100, kw.get("Y", 0x1000), 80, 8, None, None, kw.get("p", 1.5),
        kw.get("eps", 0.0), kw.get("tau", 1e-3), kw.get("it", 100), kw.get("out", out),
        kw.get("ws", 0x2000), kw.get("wsb", nb), None)
    assert call(X=None) == inv and call(out=None) == inv and call(ws=None) == inv
    assert call(p=0.5) == inv and call(eps=-1.0) == inv and call(tau=0.0) == inv and call(it=0) == inv
    assert call(wsb=nb - 1) == B.POT_ERR_NOMEM


def test_timing_enable_rejects_negative_stride():
    """pot_timing_enable(every): 0 stops, every >= 1 samples, every < 0 is
    invalid (no device work either way while nothing was timed)."""
    lib = P.lib()
    assert lib.pot_timing_enable(-1) == B.POT_ERR_INVALID
    assert lib.pot_timing_enable(0) == 0
    with pytest.raises(ValueError):
        P.timing_enable(True, every=0)


def test_static_scratch_size_matches_header():
    """The binding's size of the allocation-free entry point's scratch array is
    the header's POT_STATIC_SCRATCH_BYTES, and pairs up to 32768^2 at d = 64
    fit in it."""
    import re
    txt = B.HEADER.read_text()
    m = re.search(r"#define POT_STATIC_SCRATCH_BYTES \((\d+)u << (\d+)\)", txt)
    assert m and int(m.group(1)) << int(m.group(2)) == B.STATIC_SCRATCH_BYTES
    assert P.lib().pot_sinkhorn_divergence_bytes(32768, 32768, 64) <= B.STATIC_SCRATCH_BYTES
    assert P.lib().pot_sinkhorn_divergence_bytes(70000, 70000, 64) > B.STATIC_SCRATCH_BYTES


def test_noalloc_divergence_rejects_invalid_arguments_on_the_host():
    out = (C.c_double * 5)()
    L = P.lib()
    # null inputs, d out of range, negative eps, tau <= 0, max_iter < 1: all before any HIP call
    assert L.pot_sinkhorn_divergence_noalloc(None, 10, None, 10, 4, None, None, 0.0, 1e-3, 10, out,
                                             None) == B.POT_ERR_INVALID
    fake = C.c_void_p(0x1000)
    assert L.pot_sinkhorn_divergence_noalloc(fake, 10, fake, 10, 300, None, None, 0.0, 1e-3, 10,
                                             out, None) == B.POT_ERR_INVALID
    assert L.pot_sinkhorn_divergence_noalloc(fake, 10, fake, 10, 4, None, None, -1.0, 1e-3, 10,
                                             out, None) == B.POT_ERR_INVALID
    assert L.pot_sinkhorn_divergence_noalloc(fake, 10, fake, 10, 4, None, None, 0.0, 0.0, 10,
                                             out, None) == B.POT_ERR_INVALID
    assert L.pot_sinkhorn_divergence_noalloc(fake, 10, fake, 10, 4, None, None, 0.0, 1e-3, 0,
                                             out, None) == B.POT_ERR_INVALID
    # too large for the scratch: refused before any HIP call
    assert L.pot_sinkhorn_divergence_noalloc(fake, 70000, fake, 70000, 64, None, None, 0.0, 1e-3,
                                             10, out, None) == B.POT_ERR_NOMEM
