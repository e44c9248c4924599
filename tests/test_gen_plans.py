"""Host-side checks of the kernel generator's per-class plans (no GPU, no
compilation): the staged pass plans cover every contraction target exactly
once within the configured pass size, every staged class fits its waves per
SIMD, and the digestion groups are at least one output wide."""
import importlib.util
import os

import pytest

_GEN = os.path.join(os.path.dirname(__file__), "..", "paper_1905_01381_amd", "csrc", "gen_eri.py")


@pytest.fixture(scope="module")
def gen():
    spec = importlib.util.spec_from_file_location("gen_eri_plans", _GEN)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_staged_passes_partition_targets(gen):
    for cls, (cap, waves) in gen.STAGE_CFG.items():
        es, fs = gen.targets(*cls)
        want = sorted((e, f) for e in es for f in fs)
        plan = gen.stage_subsets(*cls)
        got = sorted(t for p in plan for t in p)
        assert got == want, cls
        assert all(0 < len(p) <= cap for p in plan), cls
        assert waves in (1, 2), cls


def test_pass_plans_cost_no_more_than_fixed_blocks(gen):
    """The chosen plan re-runs no more VRR work (plus per-pass overhead) than
    cutting the target list into consecutive blocks of the same size."""
    for cls, (cap, _) in gen.STAGE_CFG.items():
        es, fs = gen.targets(*cls)
        flat = [(e, f) for e in es for f in fs]
        blocks = [flat[i:i + cap] for i in range(0, len(flat), cap)]
        plan = gen.stage_subsets(*cls)
        cost = gen._pass_cost(*cls, plan) + gen.PASS_OVERHEAD * len(plan)
        base = gen._pass_cost(*cls, blocks) + gen.PASS_OVERHEAD * len(blocks)
        assert cost <= base, cls


def test_single_pass_is_the_lower_bound(gen):
    for cls in gen.STAGE_CFG:
        es, fs = gen.targets(*cls)
        one = gen._pass_cost(*cls, [[(e, f) for e in es for f in fs]])
        assert gen._pass_cost(*cls, gen.stage_subsets(*cls)) >= one, cls


def test_wave_minimums_and_digest_groups(gen):
    for cls, w in gen.UNSTAGED_WAVES.items():
        assert not gen.is_staged(*cls) and w >= 2, cls
        assert gen.waves_per_simd(*cls) == w
    for cls in gen.DIGEST_VALUES_CLASS:
        assert gen.is_staged(*cls), cls
    assert gen.DIGEST_VALUES >= 1 and all(v >= 1 for v in gen.DIGEST_VALUES_CLASS.values())
