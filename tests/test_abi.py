"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/osm.h declares, sizes its footprint on the host and rejects bad
arguments before touching the GPU."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    txt = open(os.path.join(ROOT, "include", "osm.h")).read()
    return sorted(set(re.findall(
        r"^\s*(?:osm_status|void|const char \*|int32_t)\s*(osm_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ["osm_query", "osm_setup", "osm_factor", "osm_step", "osm_interface_apply",
              "osm_set_interface_guess", "osm_get_interface", "osm_destroy", "osm_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1603_05110_amd import osm
    lib = osm.load_library()
    for n in declared():
        assert hasattr(lib, n), n
    assert sorted(osm.EXPORTS) == declared()


def _pb(**kw):
    from workloads import Problem, equal_strips
    base = dict(xl=-1.0, xr=1.0, yb=-1.0, yu=1.0, ncx=16, ncy=8, nsub=2,
                strip_cells=equal_strips(16, 2), lap_coef=1.0, beta=1.0, p=1.0, p_bc=1.0,
                dt=0.01)
    base.update(kw)
    return Problem(**base)


def test_query_footprint_scales_with_the_factor():
    from paper_1603_05110_amd import osm
    d1, _ = osm.osm_query(_pb(ncy=256))
    d2, _ = osm.osm_query(_pb(ncy=512))
    # dominated by (ncx + nsub) dense ny x ny complex blocks
    assert d1 >= 18 * 257 * 257 * 16
    assert 3.0 < d2 / d1 < 4.5
    dc, _ = osm.osm_query(_pb(ncy=512), prec="c32")
    assert dc < d2


@pytest.mark.parametrize("kw", [dict(strip_cells=[10, 5]), dict(strip_cells=[15, 1]),
                                dict(p=0.0), dict(nsub=1, strip_cells=[16]), dict(dt=-1.0)])
def test_invalid_problems_are_rejected_on_the_host(kw):
    from paper_1603_05110_amd import osm
    with pytest.raises(osm.OsmError) as e:
        osm.osm_query(_pb(**kw))
    assert e.value.status == osm.OSM_EINVAL


def test_setup_reports_enomem_before_allocating():
    """The paper's preconditioner ran out of memory at N = 128; here the
    footprint check runs first and returns ENOMEM (host-forced with a cap)."""
    import ctypes
    from paper_1603_05110_amd import osm
    prob, keep = osm.make_problem(_pb(ncy=64))
    opt = osm.make_options(mem_cap=1024)
    h = ctypes.c_void_p()
    st = osm._lib.osm_setup(ctypes.byref(prob), ctypes.byref(opt), None, ctypes.byref(h))
    assert st == osm.OSM_ENOMEM
    assert not h.value
    assert b"exceeds" in osm._lib.osm_last_error(None)


def test_batch_footprint_is_the_sum_of_its_instances():
    from paper_1603_05110_amd import osm
    pbs = [_pb(ncy=32), _pb(ncx=24, ncy=48, nsub=3, strip_cells=[6, 8, 10])]
    # a lone instance of these sizes keeps half-storage factors and adds the
    # solve's partial buffer (nsub x 2 x 64 x 2 x ny complex128); batched
    # instances keep full storage and do not
    part = sum(pb.nsub * 2 * 64 * 2 * (pb.ncy + 1) * 16 for pb in pbs)
    single = sum(osm.osm_query(pb)[0] for pb in pbs) - part
    dev, _ = osm.osm_query_batch(pbs)
    assert single < dev < single + 64 * 1024


def test_batch_rejects_bad_arguments_on_the_host():
    from paper_1603_05110_amd import osm
    with pytest.raises(osm.OsmError) as e:
        osm.osm_query_batch([_pb(beta=0.0), _pb(beta=0.0)], algo="interface")
    assert e.value.status == osm.OSM_EUNSUPPORTED
    with pytest.raises(osm.OsmError) as e:
        osm.osm_query_batch([_pb(), _pb()], algo="precond", krylov="bicgstab", gmres_restart=8)
    assert e.value.status == osm.OSM_EINVAL
    # preconditioned batches: every instance's L_h in the footprint
    dc, _ = osm.osm_query_batch([_pb(), _pb()])
    dp, _ = osm.osm_query_batch([_pb(), _pb()], algo="precond")
    assert dp > dc
    with pytest.raises(osm.OsmError) as e:
        osm.osm_query_batch([_pb(), _pb(strip_cells=[10, 5])])
    assert e.value.status == osm.OSM_EINVAL
    assert b"instance 1" in osm._lib.osm_last_error(None)
    import ctypes
    opt = osm.make_options()
    fp = osm.osm_footprint()
    assert osm._lib.osm_query_batch(None, 0, ctypes.byref(opt), ctypes.byref(fp)) == osm.OSM_EINVAL


def test_batch_setup_reports_enomem_before_allocating():
    import ctypes
    from paper_1603_05110_amd import osm
    arr, keep = osm._problem_array([_pb(ncy=64), _pb(ncy=32)])
    opt = osm.make_options(mem_cap=4096)
    h = ctypes.c_void_p()
    st = osm._lib.osm_setup_batch(arr, 2, ctypes.byref(opt), None, ctypes.byref(h))
    assert st == osm.OSM_ENOMEM
    assert not h.value


def test_guess_options_and_network_arguments_are_checked_on_the_host():
    import ctypes
    from paper_1603_05110_amd import osm
    with pytest.raises(osm.OsmError) as e:
        osm.osm_query(_pb(), guess=4)
    assert e.value.status == osm.OSM_EINVAL
    h = ctypes.c_void_p()
    assert osm._lib.osm_net_create(0, None, ctypes.byref(h)) == osm.OSM_EINVAL
    assert not h.value
    from oracle import nn
    assert osm.NET_NPARAMS == nn.NPARAM


@pytest.mark.parametrize("kw", [dict(q_estimate=2), dict(q_estimate=-1), dict(solve_shape=9),
                                dict(g1_init=2), dict(g1_init=-1), dict(krylov_code=2),
                                dict(algo="interface"),
                                dict(algo="precond", krylov="bicgstab", gmres_restart=3)])
def test_solver_switches_are_checked_on_the_host(kw):
    """Out-of-range values of the solver switches are rejected by osm_query
    (EINVAL) before any device work: the inner stopping test, the solve
    shape, the first interface vector, the Krylov solver of P (BiCGStab
    needs room for its work vectors), and the interface Krylov algorithm on
    a nonlinear problem (beta != 0)."""
    import ctypes
    from paper_1603_05110_amd import osm
    if "krylov_code" in kw:
        prob, keep = osm.make_problem(_pb())
        opt = osm.make_options()
        opt.krylov = kw["krylov_code"]
        fp = osm.osm_footprint()
        st = osm._lib.osm_query(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(fp))
        assert st == osm.OSM_EINVAL
        return
    with pytest.raises(osm.OsmError) as e:
        osm.osm_query(_pb(), **kw)
    assert e.value.status == osm.OSM_EINVAL


def test_interface_krylov_is_accepted_for_the_linear_problem():
    from paper_1603_05110_amd import osm
    d, _ = osm.osm_query(_pb(beta=0.0), algo="interface")
    dc, _ = osm.osm_query(_pb(beta=0.0))
    dp, _ = osm.osm_query(_pb(beta=0.0), algo="precond")
    assert dc < d < dp      # a Krylov basis, but no L_h


def test_options_struct_matches_the_header():
    """The ctypes mirror of osm_options ends with g1_init, seed, krylov and
    strip_order, laid out
    as the C compiler lays out include/osm.h (checked with the C compiler
    of the build)."""
    import ctypes
    import shutil
    import subprocess
    import tempfile
    from paper_1603_05110_amd import osm
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = (
        '#include <stddef.h>\n#include <stdio.h>\n#include "osm.h"\n'
        'int main(void) { printf("%zu %zu %zu %zu %zu\\n", sizeof(osm_options), '
        'offsetof(osm_options, g1_init), offsetof(osm_options, seed), '
        'offsetof(osm_options, krylov), sizeof(osm_problem)); '
        'printf("%zu %zu\\n", offsetof(osm_options, strip_order), offsetof(osm_options, lh_form)); '
        'printf("%zu %zu\\n", sizeof(osm_step_stats), offsetof(osm_step_stats, guess_ratio)); '
        'return 0; }\n')
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.run([cc, "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    size, off_g1, off_seed, off_kr, psize, off_so, off_ld, ssize, off_gr = map(int, out)
    assert off_so == osm.osm_options.strip_order.offset
    assert off_ld == osm.osm_options.lh_form.offset
    assert ssize == ctypes.sizeof(osm.osm_step_stats)
    assert off_gr == osm.osm_step_stats.guess_ratio.offset
    assert size == ctypes.sizeof(osm.osm_options)
    assert off_g1 == osm.osm_options.g1_init.offset
    assert off_seed == osm.osm_options.seed.offset
    assert off_kr == osm.osm_options.krylov.offset
    assert psize == ctypes.sizeof(osm.osm_problem)


def test_strip_order_footprint_and_checks():
    """y-line order keeps ny nx_j^2 values per strip (complex128, or complex64
    with prec c32) instead of the
    node-line order's ny^2 per packed line; the tuned order keeps both where
    the y-line order is available, and only the node-line factor where it is
    not (S_pade^m).  The y-line order needs the Robin condition and strips of
    at most 64 node-lines, and batches use the node-line order."""
    from paper_1603_05110_amd import osm
    pb = _pb(ncy=256)
    dn, _ = osm.osm_query(pb)
    dy, _ = osm.osm_query(pb, strip_order="y")
    dt, _ = osm.osm_query(pb, strip_order="tuned")
    ny, lt = 257, 18
    node_factor = lt * ny * ny * 16
    y_factor = 2 * 9 * 9 * ny * 16
    assert dy < dn - node_factor + y_factor + 64 * 1024
    assert dt >= dn + y_factor
    # complex-FP32 storage halves the y-line inverses
    dy32, _ = osm.osm_query(pb, strip_order="y", prec="c32")
    assert dy - dy32 >= y_factor // 2 - 64 * 1024 and dy32 < dy
    pade = _pb(ncy=32, tc="pade", pade_m=4, p=0.0, p_bc=0.0)
    assert osm.osm_query(pade, strip_order="tuned")[0] == osm.osm_query(pade)[0]
    for bad in [dict(pb=pade), dict(pb=_pb(ncx=200, strip_cells=[100, 100]))]:
        with pytest.raises(osm.OsmError) as e:
            osm.osm_query(bad["pb"], strip_order="y")
        assert e.value.status == osm.OSM_EINVAL
    # a strip wider than 64 node-lines: the tuned order falls back to node-line
    wide = _pb(ncx=200, strip_cells=[100, 100])
    assert osm.osm_query(wide, strip_order="tuned")[0] == osm.osm_query(wide)[0]
    with pytest.raises(osm.OsmError) as e:
        osm.osm_query_batch([_pb(), _pb()], strip_order="y")
    assert e.value.status == osm.OSM_EINVAL
    import ctypes
    prob, keep = osm.make_problem(pb)
    opt = osm.make_options()
    opt.strip_order = 3
    fp = osm.osm_footprint()
    assert osm._lib.osm_query(ctypes.byref(prob), ctypes.byref(opt),
                              ctypes.byref(fp)) == osm.OSM_EINVAL
