"""Host logic of bench.py: the kernel-class patterns that attribute profiler
rows (rocprofv3 kernel names) to the four classes of the 2D step, and the
source hash that ties the stored counter results to the kernel sources."""
import importlib.util
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


# kernel names as the profiler prints them, by class (default strip form,
# the column tiles and the Step 2 direct-source x-lines)
NAMES = {
    "rhs_e": ["void c4m::k_xlines<0, true>(c4m::XArgs, c4m::Coef, c4m::PadeTaps, c4m::YbandArgs)",
              "void c4m::k_xlines<1, true>(c4m::XArgs, c4m::Coef, c4m::PadeTaps, c4m::YbandArgs)",
              "void c4m::k_xlines<0, false>(c4m::XArgs, c4m::Coef, c4m::PadeTaps, c4m::YbandArgs)"],
    "solve_e": ["void c4m::k_strip<5, 0, 8, 1, 3>(c4m::ColArgs, c4m::Coef, c4m::PadeLine)",
                "void c4m::k_strip<5, 1, 16, 1, 3>(c4m::ColArgs, c4m::Coef, c4m::PadeLine)",
                "void c4m::k_col<5, 0, c4m::TileShape<128, 4>, 0>(c4m::ColArgs)"],
    "rhs_h": ["void c4m::k_xlines<2, false>(c4m::XArgs, c4m::Coef, c4m::PadeTaps, c4m::YbandArgs)",
              "void c4m::k_xlines<3, false>(c4m::XArgs, c4m::Coef, c4m::PadeTaps, c4m::YbandArgs)"],
    "solve_h": ["void c4m::k_strip_h<5, 2, 8, 1, 3>(c4m::ColArgs, c4m::ColArgs, c4m::Coef)",
                "void c4m::k_strip<5, 3, 16, 1, 3>(c4m::ColArgs, c4m::Coef, c4m::PadeLine)",
                "void c4m::k_strip<5, 4, 16, 1, 3>(c4m::ColArgs, c4m::Coef, c4m::PadeLine)",
                "void c4m::k_col<5, 4, c4m::TileShape<128, 4>, 0>(c4m::ColArgs)"],
}
OTHERS = ["c4m::k_lap_convert(double*, double const*)", "c4m::k_zero_walls(double*)",
          "__amd_rocclr_fillBufferAligned", "void c4m::k_term3<0, 1>(c4m::Term3, double)",
          "void c4m::k_cheb3t<double, double, double, false, 0>(c4m::Cheb3T<double, double>)"]


def test_class_patterns_attribute_each_kernel_to_one_class():
    b = _bench()
    pats = {c: re.compile(p) for c, p in b.CLASS_PATTERNS.items()}
    assert set(pats) == set(NAMES)
    for cls, names in NAMES.items():
        for name in names:
            hits = [c for c, rx in pats.items() if rx.search(name)]
            assert hits == [cls], (name, hits)
    for name in OTHERS:
        assert not any(rx.search(name) for rx in pats.values()), name


BATCH_NAMES = {
    "rhs_e": ["void c4m::k_batch_stage<5, true, 0>(c4m::BatchProb const*, c4m::Sched, c4m::Coef)",
              "void c4m::k_batch_x<1>(c4m::BatchProb const*, c4m::Sched, int, c4m::Coef, c4m::PadeTaps)",
              "void c4m::k_batch_xstage<true, 0>(c4m::BatchProb const*, c4m::Sched, c4m::Coef, c4m::PadeTaps)"],
    "solve_e": ["void c4m::k_batch_stage<5, false, 1>(c4m::BatchProb const*, c4m::Sched)",
                "void c4m::k_batch_col<5, 0, c4m::TileShape<128, 2>, 0>(c4m::BatchProb const*)"],
    "rhs_h": ["void c4m::k_batch_stage<6, true, 2>(c4m::BatchProb const*, c4m::Sched)",
              "void c4m::k_batch_x<2>(c4m::BatchProb const*, c4m::Sched, int, c4m::Coef, c4m::PadeTaps)",
              "void c4m::k_batch_xstage<false, 2>(c4m::BatchProb const*, c4m::Sched, c4m::Coef, c4m::PadeTaps)"],
    "solve_h": ["void c4m::k_batch_stage<5, true, 3>(c4m::BatchProb const*, c4m::Sched)",
                "void c4m::k_batch_col<5, 4, c4m::TileShape<64, 4>, 0>(c4m::BatchProb const*)",
                "void c4m::k_batch_col<5, 2, c4m::TileShape<128, 2>, 1>(c4m::BatchProb const*)"],
    "step": ["void c4m::k_batch_step<5, true>(c4m::BatchProb const*, c4m::Sched, c4m::Coef)"],
}


def test_batch_class_patterns_attribute_each_kernel_to_one_class():
    b = _bench()
    pats = {c: re.compile(p) for c, p in b.BATCH_CLASS_PATTERNS.items()}
    assert set(pats) == set(BATCH_NAMES)
    for cls, names in BATCH_NAMES.items():
        for name in names:
            hits = [c for c, rx in pats.items() if rx.search(name)]
            assert hits == [cls], (name, hits)
    for name in OTHERS + [n for v in NAMES.values() for n in v]:
        assert not any(rx.search(name) for rx in pats.values()), name


NAMES_3D = {
    "rhs": ["void c4m::k_condition3<1>(c4m::Term3, double)",
            "void c4m::k_term3<0, 0>(c4m::Term3, double, c4m::PadeTaps, c4m::PadeLine)",
            "void c4m::k_march3<1, 0>(c4m::Term3, double, c4m::PadeTaps, c4m::PadeLine, int)",
            "void c4m::k_march3<2, 0>(c4m::Term3, double, c4m::PadeTaps, c4m::PadeLine, int)"],
    "solve": ["void c4m::k_cheb3t<double, double, double, false, 0>(c4m::Cheb3T<double, double>)",
              "void c4m::k_cheb3t<double, double, double, true, 1>(c4m::Cheb3T<double, double>)"],
}


def test_3d_class_patterns_attribute_each_kernel_to_one_class():
    b = _bench()
    pats = {c: re.compile(p) for c, p in b.CLASS_PATTERNS_3D.items()}
    assert set(pats) == set(NAMES_3D) == set(b.CALLS_3D)
    for cls, names in NAMES_3D.items():
        for name in names:
            hits = [c for c, rx in pats.items() if rx.search(name)]
            assert hits == [cls], (name, hits)
    others = OTHERS[:3] + [n for v in NAMES.values() for n in v]
    for name in others:
        assert not any(rx.search(name) for rx in pats.values()), name


def test_source_hash_is_stable_and_hex():
    b = _bench()
    h = b.kernel_source_hash()
    assert h == b.kernel_source_hash()
    assert re.fullmatch(r"[0-9a-f]{16}", h)
