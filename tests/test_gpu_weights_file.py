"""anon_model_load on the GPU: a model loaded from its weights file gives the
same logits, bit for bit, as the model created from the same host array."""
import numpy as np
import pytest

import synth
from synth.configs import TINY
from tests.gpu_common import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_loaded_model_equals_created_model(tmp_path, precision):
    import torch
    from paper_2606_15650_amd import api
    from paper_2606_15650_amd.pipeline import DeviceBatch, Pipeline
    W = synth.make_weights(TINY, 5)
    blob = synth.weights_blob(TINY, W)
    path = str(tmp_path / "tiny.anonw")
    api.write_weights(path, TINY, blob)
    rb = synth.generate_records(20, ("uniform", 16, 128), TINY.n_types, TINY.vocab, 9)
    outs = []
    for m in (api.Model(TINY, blob, precision), api.Model.load(path, TINY, precision)):
        lab, z, mg = Pipeline(m).ner(DeviceBatch(rb), logits=True)
        torch.cuda.synchronize()
        outs.append(z[:rb.n_tokens].cpu().numpy())
        m.close()
    say(f"[weights file] {precision}: {rb.n_tokens} tokens")
    assert np.array_equal(outs[0], outs[1])
    with pytest.raises(api.AnonError):  # the caller's config must match the file's
        from synth.configs import ModelConfig
        api.Model.load(path, ModelConfig(n_layers=3, hidden=128, n_heads=2, ffn=512, vocab=8192, n_labels=9),
                       precision)
