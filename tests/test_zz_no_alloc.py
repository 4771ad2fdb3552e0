"""ulppm_forces_static, the entry point that allocates no device memory,
against ulppm_forces with a context of the same family capacity: two calls
in a row on the one static scratch array, the second with a smaller input,
each checked against the context's result at the FP64 bar (1e-11 relative;
the kernels are the same, so the results are expected to be equal): the
conjugate force state in FP64 and mixed precision, Eq. 51 in FP64."""
import sys

import numpy as np
import pytest

from paper_2203_05562_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _state(gpu, dims, seed, vscale):
    from paper_2203_05562_amd.ulppm import column_state
    col = inputs.make_column(inputs.CONFIGS["C0"], seed=seed, dims=dims)
    G = column_state(col)
    prm = gpu.make_params(col["params"])
    ctx = gpu.Context(col["n"], max_family=gpu.STATIC_MAX_FAMILY)
    ctx.init_state(G, prm, col["params"]["ocr"])
    prm.dt = 0.5 * ctx.dt_crit(G, prm)
    import torch
    v = inputs.random_velocity(col["n"], seed + 50, vscale)
    v[col["fixed"] == 1] = 0.0
    G["v"].copy_(torch.from_numpy(np.ascontiguousarray(v.T)))
    return G, prm, ctx


def test_forces_static_matches_forces():
    import torch
    assert torch.cuda.is_available()
    from paper_2203_05562_amd import ulppm as gpu
    gpu.load_library()
    for dims, seed, vscale in (((8, 8, 16), 3, 0.3), ((6, 6, 9), 4, 0.1)):
        say("forces_static", dims, seed)
        G, prm, ctx = _state(gpu, dims, seed, vscale)
        # the conjugate force state in both precisions, and Eq. 51 in FP64,
        # whose own force-state sums also sit in the scratch array
        for precision, mode in ((gpu.ULPPM_FP64, gpu.ULPPM_FORCE_CONJUGATE), (gpu.ULPPM_MIXED, gpu.ULPPM_FORCE_CONJUGATE),
                                (gpu.ULPPM_FP64, gpu.ULPPM_FORCE_EQ51)):
            prm.precision = precision
            prm.force_mode = mode
            f_ref, T_ref, rep_ref = ctx.forces(G, prm, prm.dt, want_T=True)
            nb = rep_ref["n_bonds"]
            f = torch.full((3, G.n), np.nan, dtype=torch.float64, device="cuda")
            T = torch.full((3, nb), np.nan, dtype=torch.float64, device="cuda")
            rep = gpu.forces_static(G, prm, prm.dt, f, T)
            torch.cuda.synchronize()
            for k in ("n_bonds", "n_tests", "n_triples", "n_degenerate", "n_plastic"):
                assert rep[k] == rep_ref[k], (k, rep[k], rep_ref[k])
            fa, fr = f.cpu().numpy(), f_ref.cpu().numpy()
            Ta, Tr = T.cpu().numpy(), T_ref.cpu().numpy()
            ef = np.linalg.norm(fa - fr) / np.linalg.norm(fr)
            eT = np.abs(Ta - Tr).max() / np.abs(Tr).max()
            say("  precision", precision, "force mode", mode, "f rel", ef, "T max rel", eT, "bonds", nb,
                "max family", rep_ref["max_family"])
            assert ef <= 1e-11 and eT <= 1e-11
        ctx.close()


def test_forces_static_rejects_sizes_beyond_its_array():
    from paper_2203_05562_amd import ulppm as gpu
    col = inputs.make_column(inputs.CONFIGS["C0"], dims=(16, 16, 9))
    assert col["n"] > gpu.STATIC_MAX_POINTS
    from paper_2203_05562_amd.ulppm import column_state
    G = column_state(col)
    import torch
    f = torch.zeros((3, G.n), dtype=torch.float64, device="cuda")
    with pytest.raises(gpu.UlppmError) as ei:
        gpu.forces_static(G, gpu.make_params(col["params"]), 0.0, f)
    assert ei.value.code == -1
