"""GPU tests of the patch-sweep variants and their autotuner through the
C-ABI: on every level and for both patch forms (complex time-diagonal 21x21
and real 42x42), every variant computes the additive Vanka step of variant
0 (they differ in workgroup size, loads in flight and rows per lane, i.e.
only in the summation order inside a patch: 1e-13 relative in FP64, 1e-5 in
FP32), and the autotuner keeps the variant with the smallest measured time."""
import pytest

from paper_2603_28706_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2603_28706_amd import pnsmg  # noqa: E402

MODEL = dict(p=1.5, delta=1e-2, nu=1.0, nu_inf=1e-3, gamma1=40.0, gamma2=40.0, sigma_max=1.0,
             convection=1, qsign=1, lin=pnsmg.MODIFIED_NEWTON)


@pytest.mark.parametrize("kind", [pnsmg.PATCH_SURROGATE, pnsmg.PATCH_EXACT])
@pytest.mark.parametrize("precision,tol", [(pnsmg.FP64, 1e-13), (pnsmg.FP32, 1e-5)])
def test_every_sweep_variant_computes_the_same_step(kind, precision, tol):
    n = (48, 32)
    ctx = pnsmg.Context(n, n_levels=3, precision=precision)
    ctx.pns_set_patch_kind(kind)
    uk = inputs.uniform(601, 2 * ctx.sizes()["nv"])
    ctx.pns_set_state(MODEL, torch.tensor(uk, device="cuda"))
    masks = pnsmg.masks_to_bits(inputs.truncation_masks(n, seed=602))
    ctx.pns_vanka_setup(masks)
    for level in range(3):
        info = ctx.pns_sweep_variant(level)
        times = [ctx.pns_sweep_variant_time(level, v) for v in range(info["count"])]
        assert all(t > 0 for t in times)
        assert times[info["variant"]] == min(times)
        nst = ctx.sizes(level)["nst"]
        r = torch.tensor(inputs.uniform(603 + level, nst), dtype=ctx.dtype, device="cuda")
        outs = []
        for v in range(info["count"]):
            ctx.pns_set_sweep_variant(level, v)
            d = ctx.vector(level)
            ctx.pns_vanka_smooth(level, 1, 0.3, r, d)
            outs.append(d.double())
        torch.cuda.synchronize()
        ref = outs[0]
        for v, o in enumerate(outs):
            err = float(torch.linalg.norm(o - ref) / torch.linalg.norm(ref))
            assert err <= tol, (level, v, err)
        print(f"kind={kind} prec={precision} level={level}: autotuned {info}, "
              f"times {[round(t, 4) for t in times]} ms")
