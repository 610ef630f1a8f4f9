"""The allocation-free energy measurement (hsg_measure_energy_static) against
hsg_measure_energy, through the C-ABI: the same kernels with the partial sums
in the library's fixed device array instead of the caller's scratch, so the
energies agree bit for bit. Two calls in a row, the second on a smaller
problem (the fixed array keeps the first call's partials, which the second
must overwrite); a third on a three-size batch with a field."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from paper_1204_6192_amd import inputs  # noqa: E402


def test_static_energy_matches_the_scratch_version():
    from paper_1204_6192_amd import hsg
    big = inputs.make_instance("batched", scale_samples=8, L_override=16)
    rng = np.random.Generator(np.random.Philox(inputs.INSTANCE_SEED_BASE + 70))
    small = [inputs.make_group(rng, 6, 1, 2, inputs.geometric_ladder(0.1, 0.3, 3))]
    mixed = []
    for L, D, field in ((8, 2, ("gaussian", 0.2)), (12, 1, None), (20, 2, ("gaussian", 0.1))):
        mixed.append(inputs.make_group(rng, L, D, 2, inputs.geometric_ladder(0.1, 0.3, 4), field=field,
                                       sample_uid_base=len(mixed) * 4))
    for groups, storage in ((big.groups, "f32"), (small, "f32"), (mixed, "f16")):
        lat = hsg.Lattice(groups, seed=big.seed, storage=storage)
        lat.sweep(2)
        want = lat.measure_energy()
        got = torch.full_like(want, float("nan"))
        hsg.check(hsg.lib.hsg_measure_energy_static(lat.h, got.data_ptr(),
                                                    torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
        assert torch.equal(got, want), (groups[0].L, storage)
        # the energies the next tempering pass uses are the measured ones
        assert torch.equal(lat.get_energies(), want)
        lat.close()


def test_static_energy_rejects_a_null_output():
    """A NULL output is rejected before anything is launched. (The 16 MiB limit
    needs over 2^30 sites of spins to reach, about 4 GiB even at 4 bytes per
    spin, so it is not exercised here.)"""
    from paper_1204_6192_amd import hsg
    rng = np.random.Generator(np.random.Philox(inputs.INSTANCE_SEED_BASE + 71))
    g = inputs.make_group(rng, 8, 1, 1, inputs.geometric_ladder(0.1, 0.3, 1))
    lat = hsg.Lattice([g], seed=1)
    with pytest.raises(hsg.HSGError) as ei:
        hsg.check(hsg.lib.hsg_measure_energy_static(lat.h, None, None))
    assert ei.value.status == hsg.E_INVALID
    lat.close()
