"""igafd_features_noalloc (the variant for callers that cannot allocate)
against igafd_features: two calls in a row on one GPU, the second on a
smaller problem, so that the static accumulator holds the first call's
contents when the second starts; the outputs must be equal bit for bit (the
same kernels in the same order) and match the oracle's features.  A problem
above the accumulator's limit is refused by the host-side size check."""
import numpy as np
import pytest

import synth
from helpers import to_host
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def test_features_noalloc_matches_features():
    import torch

    import paper_1602_01636_amd as api
    api.lib()
    probs = [synth.uniform_problem(3, [14, 12, 16], 4, geometry=synth.warped_geometry(6),
                                   coefficient=synth.sincos_coefficient(0.4, 1, 2, 0.3, 0.1)),
             synth.uniform_problem(3, [6, 7, 5], 2, geometry={"kind": "ring"})]
    for k, prob in enumerate(probs):
        print(f"noalloc features: problem {k}", flush=True)
        with api.igafd_setup(prob) as ctx:
            ref = torch.empty(ctx.N * 8, dtype=torch.float32, device="cuda")
            out = torch.full((ctx.N * 8,), float("nan"), dtype=torch.float32, device="cuda")
            api.igafd_features(ctx, ref)
            api.igafd_features_noalloc(ctx, out)
            torch.cuda.synchronize()
            assert torch.equal(ref, out), k
            np.testing.assert_allclose(to_host(out).reshape(-1, 8), omlp.features(prob), rtol=2e-6, atol=2e-7)
    # a context that assembled its features with A: the variant copies them
    with api.igafd_setup(probs[1], features=True) as ctx:
        out = torch.full((ctx.N * 8,), float("nan"), dtype=torch.float32, device="cuda")
        api.igafd_features_noalloc(ctx, out)
        np.testing.assert_allclose(to_host(out).reshape(-1, 8), omlp.features(probs[1]), rtol=2e-6, atol=2e-7)
    # N = 102^3 > 2^20: refused before any launch
    with api.igafd_setup(synth.uniform_problem(3, 103, 1)) as ctx:
        assert ctx.N > 1 << 20
        out = torch.empty(ctx.N * 8, dtype=torch.float32, device="cuda")
        with pytest.raises(api.IgafdError, match="static accumulator"):
            api.igafd_features_noalloc(ctx, out)
