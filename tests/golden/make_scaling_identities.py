"""Writes scaling_identities.json: closed forms of a one-qubit angle embedding followed by a Z
readout, <Z> = cos(theta) for RX(theta)|0> and RY(theta)|0> alike, composed with the input
scalings of eq. scale (section "QPINN architecture and ansatz designs").

* acos and asin: the caption of the input-scaling figure states them: theta = arccos(a) gives
  <Z> = a, theta = arcsin(a) + pi/2 gives <Z> = -a.
* bias, theta = (a + 1) pi/2: <Z> = cos(pi a/2 + pi/2) = -sin(pi a/2), d<Z>/da = -(pi/2) cos(pi a/2).
* none, theta = a: <Z> = cos(a), d<Z>/da = -sin(a).

Only these closed forms are evaluated here (no simulator is called)."""
import json
import math
import os

a = [-1.0, -0.75, -0.3, 0.0, 0.2, 0.5, 0.9, 1.0]
out = {
    "_source": "caption of the input-scaling figure and eq. scale, section 'QPINN architecture and ansatz designs'",
    "a": a,
    "acos_expect_z": a,
    "asin_expect_z": [-v for v in a],
    "bias_expect_z": [-math.sin(math.pi * v / 2) for v in a],
    "bias_dz_da": [-(math.pi / 2) * math.cos(math.pi * v / 2) for v in a],
    "none_expect_z": [math.cos(v) for v in a],
    "none_dz_da": [-math.sin(v) for v in a],
}
with open(os.path.join(os.path.dirname(__file__), "scaling_identities.json"), "w") as fh:
    json.dump(out, fh, indent=1)
