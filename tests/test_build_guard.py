"""The build keeps f16 subnormals: the 16-bit sweep orders biased integers with
half-float maxima, and integers 1..1023 are subnormal halves (Eq. 1-3 in
16-bit cells; the CPU emulation of that arithmetic is in test_kernel_emulation)."""
import pytest

from paper_2309_09609_amd import build


@pytest.mark.parametrize("flag", ["-fdenormal-fp-math=preserve-sign", "-fdenormal-fp-math=positive-zero",
                                  "-ffast-math", "-ffinite-math-only", "-fgpu-flush-denormals-to-zero"])
def test_flushing_flags_are_refused(flag):
    with pytest.raises(ValueError):
        build.check_flags([flag])


def test_default_flags_pass():
    build.check_flags(build.FLAGS)
    build.check_flags(["-fdenormal-fp-math=ieee", "-O2"])


def test_every_kernel_descriptor_preserves_f16_subnormals():
    modes = build.denormal_modes(build.FLAGS)
    assert any("k_sweep" in k for k in modes) and any("k_align" in k for k in modes)
    assert set(modes.values()) == {3}, modes


def test_the_descriptor_check_sees_a_flushing_build():
    src = [s for s in build.HIP_SOURCES if s.endswith("sw_align.hip")]
    modes = build.denormal_modes(build.FLAGS + ["-fdenormal-fp-math=preserve-sign"], sources=src)
    assert modes and set(modes.values()) == {0}
