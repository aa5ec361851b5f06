"""FP64 CPU oracle for the NER + pseudonymize path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU library never
calls it, links it or falls back to it.

It is a plain, slow, direct statement of what the path computes, in float64:

* ``encoder``  - the token-classification forward pass of a post-LN
  transformer encoder (the paper's stage 2 NER model, Sec. II), plus the
  reduced-precision reading that rounds where the GPU path rounds;
* ``spans``    - long-record windows, owner-window label merge and BIO span
  decoding (labels to byte ranges);
* ``pseudonym``- HMAC-SHA256 slugs and the ``[TYPE_slug]`` substitution
  (Sec. II, stage 3);
* ``recognizers`` - pattern recognizers beside the NER model (Sec. II,
  stage 2) and the merge of overlapping detections;
* ``fields`` - schema-aware whole-field spans without NER (configured
  ``Field: value`` lines);
* ``pipeline`` - the three composed over a packed batch of records.

It shares no code with the GPU path; the only common module is ``synth``
(seeded inputs, no method arithmetic).
"""
