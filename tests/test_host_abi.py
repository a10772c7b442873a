"""Host-only checks of libnnm (no GPU needed): the library loads and exports
every function include/nnm.h declares; descriptor validation maps each bad
input to its error code before any device use; the network-file parser; the
Lipschitz product bound against numpy's SVD; the binding fails loudly."""

import os
import re
import struct

import numpy as np
import pytest

import nnm_inputs as ni
import paper_2201_09147_amd as nnm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nnm.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(nnm.library_path()):
        from paper_2201_09147_amd import build as b
        b.build()
    return nnm.load_library()


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert {"load_siren_stack", "trace_rays", "analytic_normal", "free_siren_stack",
            "nnm_last_error"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name


def _levels():
    return nnm.levels_from_scene(ni.make_scene("stack3_512sq"))


def test_noalloc_entry_point_validates_on_the_host(lib):
    """trace_rays_noalloc refuses a null stack before touching a device."""
    import ctypes
    rc = lib.trace_rays_noalloc(None, None, ctypes.c_int64(16), None, None, None, None, None, None, None, None, None)
    assert rc == -1 and b"null" in lib.nnm_last_error()


def test_validate_accepts_workload_scenes(lib):
    for name in ["single_64x1_128sq", "stack3_512sq", "anim16_1024sq"]:
        s = ni.make_scene(name)
        for prec in ("fp32", "bf16", "fp16"):
            assert nnm.nnm_validate_stack(nnm.levels_from_scene(s), prec, s.base_sphere, s.r0, s.rho) == 0


def test_validate_error_paths(lib):
    lv = _levels()
    E = {"INVAL": -1, "FORMAT": -2, "NONFINITE": -3, "LIPSCHITZ": -4, "NESTING": -5, "UNSUPPORTED": -8}
    assert nnm.nnm_validate_stack([], "fp32") == E["INVAL"]
    bad = [nnm.LevelSpec(l.d_in, l.width, l.n_sine, l.params.copy(), l.amplitude, l.delta) for l in lv]
    bad[1].params[17] = np.nan
    assert nnm.nnm_validate_stack(bad, "fp32") == E["NONFINITE"]
    bad = list(lv)
    bad[0] = nnm.LevelSpec(3, 48, 2, lv[0].params, 0.005, 0.05)
    assert nnm.nnm_validate_stack(bad, "fp32") == E["UNSUPPORTED"]
    bad[0] = nnm.LevelSpec(5, 32, 2, lv[0].params, 0.005, 0.05)
    assert nnm.nnm_validate_stack(bad, "fp32") == E["UNSUPPORTED"]
    assert nnm.nnm_validate_stack(lv, 7) == E["UNSUPPORTED"]
    # deltas must decrease and stay positive on all but the last level
    bad = [nnm.LevelSpec(l.d_in, l.width, l.n_sine, l.params, l.amplitude, d)
           for l, d in zip(lv, [0.01, 0.05, 0.0])]
    assert nnm.nnm_validate_stack(bad, "fp32") == E["NESTING"]
    bad = [nnm.LevelSpec(l.d_in, l.width, l.n_sine, l.params, l.amplitude, d)
           for l, d in zip(lv, [0.05, 0.0, 0.0])]
    assert nnm.nnm_validate_stack(bad, "fp32") == E["NESTING"]
    # a larger amplitude breaks the Lipschitz bound; lipschitz_max = 0 disables the check
    bad = [nnm.LevelSpec(l.d_in, l.width, l.n_sine, l.params, l.amplitude * 3, l.delta) for l in lv]
    assert nnm.nnm_validate_stack(bad, "fp32") == E["LIPSCHITZ"]
    assert nnm.nnm_validate_stack(bad, "fp32", lipschitz_max=0.0) == 0
    bad = [nnm.LevelSpec(l.d_in, l.width, l.n_sine, l.params, float("inf"), l.delta) for l in lv]
    assert nnm.nnm_validate_stack(bad, "fp32") == E["NONFINITE"]
    assert "amplitude" in lib.nnm_last_error().decode()


def test_lipschitz_bound_matches_svd(lib):
    for l in ni.make_scene("stack3_512sq").levels:
        spec = nnm.levels_from_scene(type("S", (), {"levels": [l]})())[0]
        b = nnm.nnm_level_lipschitz_bound(spec, True)
        ref = 1.0 + l.amplitude * ni.lipschitz_product_bound(l.net.layers)
        assert abs(b - ref) <= 1e-9 * ref


def test_net_file_roundtrip_and_errors(lib, tmp_path):
    net = ni.siren_init(2, 3, 64, 2, 0.015)
    p = tmp_path / "net.nnmw"
    ni.write_net_file(p, net)
    d_in, width, n_sine, params = nnm.nnm_read_net_file(str(p))
    assert (d_in, width, n_sine) == (3, 64, 2)
    assert np.array_equal(params, net.flat())
    assert lib.nnm_param_count(3, 256, 3) == 132865
    raw = p.read_bytes()
    (tmp_path / "magic.nnmw").write_bytes(b"XXXX" + raw[4:])
    (tmp_path / "short.nnmw").write_bytes(raw[:-8])
    (tmp_path / "long.nnmw").write_bytes(raw + b"\0\0\0\0")
    (tmp_path / "shape.nnmw").write_bytes(raw[:8] + struct.pack("<I", 7) + raw[12:])
    for name in ("magic", "short", "long", "shape"):
        with pytest.raises(nnm.NnmError) as e:
            nnm.nnm_read_net_file(str(tmp_path / f"{name}.nnmw"))
        assert e.value.code == -2, name
    with pytest.raises(nnm.NnmError) as e:
        nnm.nnm_read_net_file(str(tmp_path / "missing.nnmw"))
    assert e.value.code == -9


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2201_09147_amd import _binding
    monkeypatch.setattr(_binding, "_lib", None)
    monkeypatch.setattr(_binding, "_LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(nnm.NnmError):
        _binding.load_library()


def test_product_path_does_not_reference_the_oracle():
    pkg = os.path.join(ROOT, "paper_2201_09147_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), f


def test_mesh_entry_points_reject_bad_arguments_before_device_use(lib):
    """nnm_mesh_extract / nnm_grid_values / neural_normal_map validate on the host."""
    import ctypes
    fake = ctypes.c_void_p(256)  # never dereferenced: every call below fails validation first
    f = ctypes.c_float
    ext = lib.nnm_mesh_extract
    assert ext(None, 8, f(-1), f(1), f(0), 0, 0, None, None, fake, None) == -1
    assert ext(fake, 8, f(-1), f(1), f(0), 0, 0, None, None, None, None) == -1
    assert ext(fake, 1, f(-1), f(1), f(0), 0, 0, None, None, fake, None) == -1
    assert ext(fake, 513, f(-1), f(1), f(0), 0, 0, None, None, fake, None) == -1
    assert "res = 513" in lib.nnm_last_error().decode()
    assert ext(fake, 8, f(1), f(-1), f(0), 0, 0, None, None, fake, None) == -1
    assert ext(fake, 8, f(-1), f(float("inf")), f(0), 0, 0, None, None, fake, None) == -1
    assert ext(fake, 8, f(-1), f(1), f(float("nan")), 0, 0, None, None, fake, None) == -1
    assert ext(fake, 8, f(-1), f(1), f(0), -1, 0, None, None, fake, None) == -1
    assert ext(fake, 8, f(-1), f(1), f(0), 4, 0, None, None, fake, None) == -1
    assert ext(fake, 8, f(-1), f(1), f(0), 0, 4, fake, None, fake, None) == -1
    assert lib.nnm_grid_values(None, 0, 8, f(-1), f(1), f(0), fake, None) == -1
    assert lib.neural_normal_map(None, 0, 4, fake, None, fake, None) == -1


def test_write_net_file_roundtrip_and_errors(lib, tmp_path):
    """nnm_write_net_file writes what nnm_read_net_file and the input module's
    reader read back; shape and count errors fail before writing."""
    net = ni.make_scene("stack3_512sq").levels[1].net
    flat = net.flat()
    p = tmp_path / "w.nnmw"
    nnm.nnm_write_net_file(str(p), net.d_in, net.width, net.n_sine, flat)
    d_in, width, n_sine, params = nnm.nnm_read_net_file(str(p))
    assert (d_in, width, n_sine) == (net.d_in, net.width, net.n_sine)
    assert np.array_equal(params, flat)
    back = ni.read_net_file(str(p))
    assert np.array_equal(back.flat(), flat)
    assert not (tmp_path / "w.nnmw.tmp").exists()
    with pytest.raises(nnm.NnmError) as e:
        nnm.nnm_write_net_file(str(tmp_path / "bad.nnmw"), net.d_in, net.width, net.n_sine, flat[:-1])
    assert e.value.code == -1
    with pytest.raises(nnm.NnmError):
        nnm.nnm_write_net_file(str(tmp_path / "bad.nnmw"), 5, net.width, net.n_sine, flat)
    with pytest.raises(nnm.NnmError) as e:
        nnm.nnm_write_net_file(str(tmp_path / "no_such_dir" / "x.nnmw"), net.d_in, net.width, net.n_sine, flat)
    assert e.value.code == -9
    assert not (tmp_path / "bad.nnmw").exists()


def _band(c, delta):
    """[|f| <= delta] for f(x) = |x| - 0.6 + c, as an interval of radii."""
    return (0.6 - c - delta, 0.6 - c + delta)


def _nested(bands):
    """Eq.(1): each band lies inside the band before it."""
    return all(bands[i - 1][0] <= bands[i][0] + 1e-15 and bands[i][1] <= bands[i - 1][1] + 1e-15
               for i in range(1, len(bands)))


def test_nesting_thresholds_prop1_and_prop2(lib):
    """Propositions 1 and 2 (Sec. 3.3) on radially offset spheres
    f_i(x) = |x| - 0.6 + c_i, whose sup differences are exact: |f_i - f_j| = |c_i - c_j|
    everywhere, and |f - f_i| = |c_i| against f = |x| - 0.6.  The bands
    [|f_i| <= delta_i] are radius intervals, so Eq.(1)'s inclusion is checked in
    closed form.  Offsets of alternating sign attain the bounds, so the thresholds
    are tight: dropping any term, or shifting an index, breaks an inclusion."""
    rng = np.random.default_rng(5)
    for m in (2, 3, 5, 8):
        for _ in range(20):
            mag = rng.uniform(0.001, 0.05, m)
            c = mag * np.where(np.arange(m) % 2 == 0, 1.0, -1.0)
            # Proposition 2: bounds against f are |c_i|
            d2 = nnm.nnm_nesting_thresholds(2, list(np.abs(c)))
            assert _nested([_band(c[i], d2[i]) for i in range(m)])
            # tight: every inclusion holds with equality at one end
            for i in range(1, m):
                lo_gap = _band(c[i], d2[i])[0] - _band(c[i - 1], d2[i - 1])[0]
                hi_gap = _band(c[i - 1], d2[i - 1])[1] - _band(c[i], d2[i])[1]
                assert min(lo_gap, hi_gap) <= 1e-15
            # Proposition 1: bounds between consecutive members are |c_i - c_{i-1}|
            sup1 = [0.0] + [abs(c[i] - c[i - 1]) for i in range(1, m)]
            d1 = nnm.nnm_nesting_thresholds(1, sup1)
            assert _nested([_band(c[i], d1[i]) for i in range(m)])
            assert d1[m - 1] == sup1[m - 1]
            # a margin raises every bound: thresholds grow, bands stay nested
            d1m = nnm.nnm_nesting_thresholds(1, sup1, 1e-3)
            assert all(a > b for a, b in zip(d1m, d1))
            assert _nested([_band(c[i], d1m[i]) for i in range(m)])
    # closed forms of the recursions for m = 3
    assert np.allclose(nnm.nnm_nesting_thresholds(2, [0.1, 0.05, 0.01]), [0.27, 0.12, 0.06], rtol=0, atol=1e-15)
    assert np.allclose(nnm.nnm_nesting_thresholds(1, [9.0, 0.05, 0.01]), [0.07, 0.02, 0.01], rtol=0, atol=1e-15)


def test_nesting_thresholds_errors(lib):
    for prop, sup, margin in [(3, [0.1, 0.1], 0.0), (1, [0.1], 0.0), (2, [0.1] * 9, 0.0),
                              (2, [0.1, -0.1], 0.0), (2, [0.1, float("nan")], 0.0), (1, [0.0, 0.1], -1.0),
                              (1, [0.0, float("inf")], 0.0)]:
        with pytest.raises(nnm.NnmError) as e:
            nnm.nnm_nesting_thresholds(prop, sup, margin)
        assert e.value.code == -1, (prop, sup, margin)
    # Proposition 1 does not read sup[0]
    assert nnm.nnm_nesting_thresholds(1, [float("nan"), 0.1]) == [0.2, 0.1]

