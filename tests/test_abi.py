"""Host-side checks of the C ABI: it loads without a GPU, exports every symbol
declared in include/hweno.h, and rejects bad arguments before any HIP call."""
import ctypes
import os
import re

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hweno.h")

h = pytest.importorskip("paper_2207_05258_amd")


def _lib_or_skip():
    if not os.path.exists(h.hweno.LIB_PATH):
        pytest.skip("libhweno.so not built")
    return h.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hweno_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("hweno_rhs", "hweno_limit", "hweno_rk3_step", "hweno_rhs_adjoint",
                     "hweno_workspace_bytes", "hweno_status_string", "hweno_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = _lib_or_skip()
    for name in declared_functions():
        assert hasattr(L, name), name


def _prob(**kw):
    base = dict(dim=2, nx=64, ny=48, physics="euler", dx=1 / 64, dy=1 / 48)
    base.update(kw)
    return h.Problem(**base)


@pytest.mark.parametrize("bad", [
    dict(dim=3),
    dict(nx=-1),
    dict(dx=0.0),
    dict(dy=-1.0),
    dict(lin_w=(0.5, 0.5, 0.1)),
    dict(lin_w=(1.0, 0.0, 0.0)),
    dict(lim_w=(0.98, 0.02, -0.0)),
    dict(lim_w=(0.9, 0.05, 0.05000001)),
    dict(eps=0.0),
    dict(cfl=-0.6),
    dict(gamma_gas=1.0),
    dict(bc_x=7),
])
def test_invalid_problems_are_rejected(bad):
    _lib_or_skip()
    with pytest.raises(h.HwenoError) as e:
        h.validate(_prob(**bad))
    assert e.value.code == 1
    assert h.workspace_bytes(_prob(**bad)) == 0


def test_reflecting_walls_are_checked_on_host():
    L = _lib_or_skip()
    ok = _prob(bc_x=h.REFLECT, bc_y=h.REFLECT).c()
    assert L.hweno_validate(ctypes.byref(ok)) == 0
    scalar = _prob(physics="burgers", bc_x=h.REFLECT).c()
    assert L.hweno_validate(ctypes.byref(scalar)) == 2          # unsupported
    assert "Euler" in L.hweno_last_error().decode()
    thin = _prob(nx=1, bc_x=h.REFLECT).c()
    assert L.hweno_validate(ctypes.byref(thin)) == 1
    thin_y = _prob(ny=1, bc_y=h.REFLECT).c()
    assert L.hweno_validate(ctypes.byref(thin_y)) == 1
    assert L.hweno_validate(ctypes.byref(_prob(nx=1, bc_y=h.REFLECT).c())) == 0


def test_characteristic_limiter_flag_is_checked():
    L = _lib_or_skip()
    c = _prob(limiter_characteristic=True).c()
    assert L.hweno_validate(ctypes.byref(c)) == 0
    c.limiter_characteristic = 2
    assert L.hweno_validate(ctypes.byref(c)) == 1
    c.limiter_characteristic = 1
    # the adjoint entry points accept the variant and run their usual checks
    assert L.hweno_rhs_adjoint(ctypes.byref(c), None, None, None, None, None, None, 0, None) == 1
    assert L.hweno_rk3_step_adjoint(ctypes.byref(c), None, None, 0, None, None, None, 0, None) == 1


def test_1d_requires_ny_one():
    L = _lib_or_skip()
    c = _prob(dim=1).c()
    c.ny = 5
    assert L.hweno_validate(ctypes.byref(c)) == 1
    c.ny = 1
    assert L.hweno_validate(ctypes.byref(c)) == 0


def test_weights_sum_tolerance():
    _lib_or_skip()
    h.validate(_prob(lin_w=(1 / 3, 1 / 3, 1 / 3), lim_w=(0.01, 0.495, 0.495)))
    h.validate(_prob(lin_w=(0.99, 0.005, 0.005)))


def test_workspace_bytes_layout():
    _lib_or_skip()
    p = _prob(nx=100, ny=30, dtype=torch.float64)
    n = 100 * 30
    need = h.workspace_bytes(p)
    # control block + two stage states (12 fields) + limited base derivatives (8 fields)
    assert need >= 128 + (2 * 12 + 8) * n * 8
    assert need < 128 + (2 * 12 + 8) * n * 8 + 4 * 256 + 256
    p32 = _prob(nx=100, ny=30, dtype=torch.float32)
    assert h.workspace_bytes(p32) < need


def test_null_pointers_and_small_workspace_are_rejected_on_host():
    L = _lib_or_skip()
    c = _prob().c()
    P = ctypes.byref(c)
    assert L.hweno_rhs(P, None, None, None, 1, None) == 1
    assert L.hweno_limit(P, None, None, None) == 1
    assert L.hweno_rk3_step(P, None, None, 0, 0.0, 0.0, None, None, None) == 1
    assert "non-NULL" in L.hweno_last_error().decode()
    # a fake (never dereferenced) pointer with a too-small workspace size
    assert L.hweno_rk3_step(P, ctypes.c_void_p(256), ctypes.c_void_p(256), 10, 0.0, 0.0,
                            None, None, None) == 3
    assert L.hweno_rk3_step(P, ctypes.c_void_p(256), ctypes.c_void_p(256), 1 << 40,
                            float("inf"), 0.0, None, None, None) == 1


def test_step_adjoint_rejects_overlapping_buffers_on_host():
    """The step adjoint writes lam and its workspace while reading state0 and the
    forward step's workspace: overlapping ranges are refused before any HIP call
    (the addresses below are never dereferenced)."""
    L = _lib_or_skip()
    c = _prob().c()
    P = ctypes.byref(c)
    swb = L.hweno_workspace_bytes(P)
    awb = L.hweno_adjoint_workspace_bytes(P)
    state_bytes = 64 * 48 * 12 * 8
    base = 1 << 40
    state0, step_ws = base, base + (1 << 34)
    ws, lam = base + (2 << 34), base + (3 << 34)
    tape = base + (4 << 34)
    vp = ctypes.c_void_p

    def call(lam_, ws_):
        return L.hweno_rk3_step_adjoint(P, vp(state0), vp(step_ws), swb, vp(tape), vp(lam_),
                                        vp(ws_), awb, None)

    assert call(state0, ws) == 1                     # lam is state0
    assert "overlap" in L.hweno_last_error().decode()
    assert call(step_ws + 256, ws) == 1              # lam inside the step workspace
    assert call(lam, lam + 256 * ((state_bytes // 2) // 256)) == 1   # ws inside lam
    assert call(lam, step_ws) == 1                   # ws is the step workspace


def test_empty_grid_is_a_noop_without_device_calls():
    L = _lib_or_skip()
    for kw in (dict(nx=0), dict(ny=0), dict(dim=1, nx=0, ny=1)):
        c = _prob(**kw).c()
        P = ctypes.byref(c)
        assert L.hweno_rhs(P, None, None, None, 1, None) == 0
        assert L.hweno_limit(P, None, None, None) == 0
        assert L.hweno_rk3_step(P, None, None, 0, 0.0, 0.0, None, None, None) == 0
        assert L.hweno_last_error().decode() == ""


def test_status_strings():
    L = _lib_or_skip()
    assert L.hweno_status_string(0).decode() == "HWENO_OK"
    assert L.hweno_status_string(3).decode() == "HWENO_ERR_WORKSPACE"
    assert L.hweno_status_string(99).decode() == "HWENO_ERR_UNKNOWN"


def test_product_package_does_not_import_the_oracle():
    import sys
    import subprocess
    code = ("import sys; import paper_2207_05258_amd; "
            "assert not any(m == 'oracle' or m.startswith('oracle.') for m in sys.modules), "
            "'oracle imported'")
    subprocess.run([sys.executable, "-c", code], check=True, cwd=ROOT)
    for dirpath, _, files in os.walk(os.path.join(ROOT, "paper_2207_05258_amd")):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f


def _edges_problem(**kw):
    import hweno_inputs as hi
    from tests import parity as P
    w = hi.double_mach(64, 16)
    return P.gpu_problem(w, torch.float64, **kw)


def test_edge_described_sides_are_checked_on_host():
    L = _lib_or_skip()
    good = _edges_problem()
    assert L.hweno_validate(ctypes.byref(good.c())) == 0
    # the binding carries every edge field into the C struct
    c = good.c()
    assert c.bc_x == h.EDGES and c.edges[3].kind[0] == h.SEG_STATE
    assert c.edges[2].kind[1] == h.SEG_REFLECT and c.edges[3].split[2] == good.edges[3].split[2]
    # scalar laws and 1D are not built with edges; both limiters are
    assert L.hweno_validate(ctypes.byref(_prob(physics="burgers", bc_x=h.EDGES,
                                                edges=good.edges).c())) == 2
    assert L.hweno_validate(ctypes.byref(_edges_problem(limiter_characteristic=True).c())) == 0
    # an obstacle needs edge-described x sides and room for the mirror images
    step = _edges_problem(obstacle=(10, 4))
    assert L.hweno_validate(ctypes.byref(step.c())) == 0
    for bad_obstacle in ((1, 4), (65, 4), (10, 0), (10, 15)):
        assert L.hweno_validate(ctypes.byref(_edges_problem(obstacle=bad_obstacle).c())) == 1
    assert L.hweno_validate(ctypes.byref(_prob(obstacle=(10, 4)).c())) == 2

    def with_edge(k, **field):
        e = good.edges[k]
        e = h.Edge(**{**dict(kind=e.kind, split=e.split, state=e.state), **field})
        return _edges_problem(edges=tuple(e if q == k else good.edges[q] for q in range(4)))
    bad = [
        with_edge(1, kind=(h.SEG_OUTFLOW, h.SEG_REFLECT)),    # copy and mirror on one side
        with_edge(0, kind=(h.SEG_STATE, 7)),
        with_edge(3, split=(0.7, float("nan"), 0.5)),
        with_edge(0, state=((1.0, 0.0, 0.0, -1.0), (1.0, 0.0, 0.0, 2.5))),   # p < 0
        with_edge(0, state=((0.0, 0.0, 0.0, 1.0), (1.0, 0.0, 0.0, 2.5))),    # rho = 0
    ]
    for p in bad:
        assert L.hweno_validate(ctypes.byref(p.c())) == 1, L.hweno_last_error().decode()
    thin = _edges_problem()
    thin.ny = 1
    assert L.hweno_validate(ctypes.byref(thin.c())) == 1        # a wall needs 2 cells across


def test_edges_are_refused_by_the_adjoint_and_batched_entry_points_on_host():
    L = _lib_or_skip()
    c = _edges_problem().c()
    assert L.hweno_adjoint_workspace_bytes(ctypes.byref(c)) == 0
    assert L.hweno_rhs_adjoint(ctypes.byref(c), None, None, None, None, None, None, 0, None) == 2
    assert L.hweno_rk3_step_adjoint(ctypes.byref(c), None, None, 0, None, None, None, 0, None) == 2
    inst = (h.hweno._CInstance * 1)()
    inst[0].nx, inst[0].ny, inst[0].dx, inst[0].dy = 64, 16, 1 / 16, 1 / 16
    inst[0].bc_x = inst[0].bc_y = h.OUTFLOW
    total = ctypes.c_int32(0)
    assert L.hweno_batch_prepare(ctypes.byref(c), inst, 1, ctypes.byref(total)) == 2
    plain = _prob().c()
    assert L.hweno_batch_prepare(ctypes.byref(plain), inst, 1, ctypes.byref(total)) == 0
    inst[0].bc_y = h.EDGES
    assert L.hweno_batch_prepare(ctypes.byref(plain), inst, 1, ctypes.byref(total)) == 2


def test_binding_structs_match_the_header_layout(tmp_path):
    """sizeof and field offsets of hweno_problem, hweno_edge and hweno_instance as a C
    compiler lays them out from include/hweno.h, against the binding's ctypes mirrors."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    fields = {
        "hweno_problem": ["dim", "nx", "ny", "physics", "dtype", "bc_x", "bc_y", "characteristic",
                          "limiter_on", "limiter_characteristic", "dx", "dy", "gamma_gas",
                          "adv_speed", "lin_w", "lim_w", "eps", "cfl", "edges", "obstacle"],
        "hweno_edge": ["kind", "split", "state"],
        "hweno_instance": ["state", "ws", "nx", "ny", "bc_x", "bc_y", "dx", "dy", "dt_fixed",
                           "t_end", "ws_bytes", "off_s1", "off_s2", "off_base", "tile_begin",
                           "n_tiles"],
    }
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "hweno.h"', 'int main(void) {']
    for st, fs in fields.items():
        src.append(f'printf("{st} size %zu\\n", sizeof({st}));')
        for f in fs:
            src.append(f'printf("{st} {f} %zu\\n", offsetof({st}, {f}));')
    src += ['return 0;', '}']
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.dirname(HEADER), str(c), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    mirrors = {"hweno_problem": h.hweno._CProblem, "hweno_edge": h.hweno._CEdge,
               "hweno_instance": h.hweno._CInstance}
    for st, cls in mirrors.items():
        assert got[(st, "size")] == ctypes.sizeof(cls), st
        for f in fields[st]:
            assert got[(st, f)] == getattr(cls, f).offset, (st, f)


def test_autotune_rejects_bad_arguments_before_any_hip_call():
    """hweno_autotune validates its batch description on the host."""
    L = _lib_or_skip()
    common = _prob(nx=1, ny=1).c()
    maps = (ctypes.c_void_p * 2)(4096, 8192)      # never dereferenced on these paths
    totals = (ctypes.c_int32 * 2)(10, 12)
    v, b = ctypes.c_int32(-1), ctypes.c_int32(-1)
    fake = ctypes.c_void_p(4096)

    def call(c=common, inst=fake, mp=maps, n=2, tot=totals, trials=2, vv=v, bb=b):
        return L.hweno_autotune(ctypes.byref(c), inst, mp, n, tot, trials, None,
                                None if vv is None else ctypes.byref(vv),
                                None if bb is None else ctypes.byref(bb), None, None)
    assert call(inst=None) == 1
    assert call(n=0) == 1
    assert call(trials=0) == 1
    assert call(trials=1001) == 1
    assert call(vv=None) == 1
    assert call(bb=None) == 1
    assert call(mp=(ctypes.c_void_p * 2)(4096, None)) == 1
    assert "variant 1" in L.hweno_last_error().decode()
    assert call(tot=(ctypes.c_int32 * 2)(10, 1)) == 1
    assert call(c=_prob(dim=1, ny=1, nx=1).c()) == 2          # batched is 2D Euler only
    assert call(c=_prob(nx=1, ny=1, eps=0.0).c()) == 1
    assert v.value == -1 and b.value == -1                    # outputs untouched on error


def test_rollout_refuses_edge_described_sides_before_stepping():
    """The differentiable rollout refuses problems its backward cannot differentiate
    before any step is taken (no GPU needed to reach the refusal)."""
    _lib_or_skip()
    edges = (h.Edge(),) * 4
    prob = _prob(nx=8, ny=8, bc_x=h.EDGES, bc_y=h.OUTFLOW, edges=edges)
    with pytest.raises(h.HwenoError) as e:
        h.Rollout.apply(torch.zeros(12, 8, 8, dtype=torch.float64), prob, 3, 0, None)
    assert e.value.code == 2 and "edge-described" in str(e.value)
