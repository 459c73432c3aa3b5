"""GPU check of the BF16 screen's tile choice: every form (256- or 128-row
blocks) and run length gives the same screened values, the same rechecked
set and the same FP64 state, bit for bit, in single steps and in the
serving engine (where requests of one d split into groups by form)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
lib = pytest.importorskip("paper_2207_06374_amd")
serve = pytest.importorskip("paper_2207_06374_amd.serve")
abi = lib._abi


def _run(n, d, steps=6, C=32, seed=3):
    s = lib.Solver(n, d, candidates=C, mode="bf16", recheck_topk=8, radius0=0.05, max_steps=10 ** 6, seed=seed)
    s.init_haar()
    reps = []
    for _ in range(steps):
        s.step()
        reps.append({k: v.clone() for k, v in s.report.items()})
    return reps, s.host_state()


@pytest.mark.parametrize("n,d", [(130, 8), (300, 16), (257, 32), (520, 64), (700, 100), (1024, 128)])
def test_every_tile_choice_gives_the_same_steps(n, d):
    ks = (2 * d + 31) // 32
    try:
        abi.set_screen_tiles([])
        ref_reps, ref_state = _run(n, d)
        forms = (0, 1) if ks <= 4 else (1,)
        for form in forms:
            for seg in (1, 2, 5, 64):
                abi.set_screen_tiles([{"ks": ks, "n_max": n, "form": form, "seg": seg}])
                reps, state = _run(n, d)
                print(f"n={n} d={d} form={form} seg={seg}", flush=True)
                for a, b in zip(reps, ref_reps):
                    for k in a:
                        assert torch.equal(a[k], b[k]), (k, form, seg)
                assert np.array_equal(state[0], ref_state[0]) and state[1:] == ref_state[1:]
    finally:
        abi.lib().trstmi_screen_tiles_set(None, 0)
        abi._install_screen_tiles(abi.lib())


def test_engine_groups_split_by_form_give_single_solve_results():
    """d = 64 requests of small N on 128-row blocks, larger N on 256-row
    blocks: two groups of the same d in one engine step."""
    reqs = [serve.Request(id=300 + k, arrival=0.0, n=n, d=64, seed=k, max_steps=16)
            for k, n in enumerate((128, 130, 400, 512))]
    try:
        abi.set_screen_tiles([{"ks": 4, "n_max": 200, "form": 1, "seg": 2},
                              {"ks": 4, "n_max": 4096, "form": 0, "seg": 3}])
        srv = serve.Server(pool_bytes=1 << 28, max_active=8, chunk=8, candidates=32, mode="bf16")
        stats = srv.run(reqs)
        srv.close()
        assert stats["done"] == 4 and stats["errors"] == 0
        abi.set_screen_tiles([])
        for r in reqs:
            F, mu, radius, step, flags = serve.solve_alone(r, candidates=32, mode="bf16", chunk=8)
            assert mu == r.mu and step == r.steps == 16, f"request {r.id}"
    finally:
        abi.lib().trstmi_screen_tiles_set(None, 0)
        abi._install_screen_tiles(abi.lib())
