"""GPU tests of snrt_stream_copy, the nontemporal device copy that bench.py uses as the
attainable read+write bandwidth: bitwise copies at sizes that end inside a grid-stride
round, and its argument checks."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2205_08417_amd import snrt
    snrt.lib()


# 16-byte vectors: 0, 1, one lane short of a block round (1023), ragged tails past one and
# past 8192 blocks' rounds, and a full state of the headline workload (198 450 x 256 floats)
@pytest.mark.parametrize("n16", [0, 1, 1023, 1025, 8192 * 1024 + 77, 198450 * 64])
def test_stream_copy_bitwise(n16):
    from paper_2205_08417_amd import snrt
    g = torch.Generator(device="cuda").manual_seed(n16 + 7)
    src = torch.randint(-2**31, 2**31 - 1, (4 * n16 + 8,), dtype=torch.int32, device="cuda",
                        generator=g)
    dst = torch.full_like(src, 0x5A5A5A5A)
    snrt.snrt_stream_copy(src, dst, 16 * n16)
    torch.cuda.synchronize()
    assert torch.equal(dst[:4 * n16], src[:4 * n16])
    # nothing written past the requested bytes
    assert bool((dst[4 * n16:] == 0x5A5A5A5A).all())


def test_stream_copy_errors():
    from paper_2205_08417_amd import snrt
    a = torch.zeros(1024, dtype=torch.float32, device="cuda")
    b = torch.zeros(1024, dtype=torch.float32, device="cuda")
    cases = [
        ((a, b, 24), snrt.SNRT_E_ARG),                       # not a multiple of 16
        ((a, b, -16), snrt.SNRT_E_ARG),
        ((None, b, 16), snrt.SNRT_E_ARG),
        ((a.data_ptr() + 4, b, 16), snrt.SNRT_E_ARG),        # misaligned source
        ((a, a.data_ptr() + 1024, 2048), snrt.SNRT_E_ALIAS),  # overlapping ranges
    ]
    for args, status in cases:
        with pytest.raises(snrt.SnrtError) as ei:
            snrt.snrt_stream_copy(*args)
        assert ei.value.status == status, args
    snrt.snrt_stream_copy(None, None, 0)   # an empty copy needs no arrays
    torch.cuda.synchronize()
