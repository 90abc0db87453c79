"""Host logic of the network backward's form (no GPU): which layers' data gradients are fused with
the ReLU' of the layer below (a run from layer 1 upward of layers at most 64 channels wide, in
BF16, with every channel count a multiple of 8), when the loss may form the last layer's dZ, and
the defaults of batched weight gradients by precision."""
import pytest

from paper_2509_24677_amd import NPVS_BF16, NPVS_F32
from paper_2509_24677_amd.train import Network


class _Shape(Network):
    """A Network's channel plan without weights or a device (the form depends on nothing else)."""

    def __init__(self, channels, dtype=NPVS_BF16):
        self.channels = list(channels)
        self.dtype = dtype

    @property
    def n_layers(self):
        return len(self.channels) - 1


@pytest.mark.parametrize("channels, fused, top_dz", [
    ([64] * 7, [False, True, True, True, True, True], True),                # the d = 4 city network
    ([512, 64, 64, 64, 64, 64, 512], [False, True, True, True, True, False], False),   # d = 8
    ([4096, 64, 64, 64, 64, 64, 4096], [False, True, True, True, True, False], False),  # d = 16
    ([8, 16, 16, 8], [False, True, True], True),                            # d = 2
    ([1, 64, 64, 64, 64, 64, 1], [False] * 6, False),                       # d = 1: 1-channel input
    ([64, 96, 64, 64], [False, False, False], False),                       # a wide layer low down
    ([64, 64, 64, 96, 64, 64], [False, True, False, False, False], False),  # the run stops below it
])
def test_fused_layers_form_a_run_from_the_first(channels, fused, top_dz):
    net = _Shape(channels)
    assert [net._fusable(i) for i in range(net.n_layers)] == fused
    assert net._chainable() == any(fused)
    assert net.loss_forms_top_dz() == top_dz


def test_defaults_by_precision():
    assert _Shape([64] * 7).backward_form() == (True, True)
    assert _Shape([64] * 7, NPVS_F32).backward_form() == (False, False)
    assert _Shape([64] * 7).backward_form(batch_wgrad=False) == (False, False)
    assert _Shape([64] * 7).backward_form(chain=False) == (True, False)
    assert _Shape([1, 64, 1]).backward_form() == (True, False)
    with pytest.raises(ValueError):
        _Shape([1, 64, 1]).backward_form(chain=True)
    assert not _Shape([64] * 7, NPVS_F32).loss_forms_top_dz()
