"""Writes scaling_identities.json: the closed forms stated in the caption of the input-scaling
figure (section "QPINN architecture and ansatz designs"): after an RX(theta) embedding and a Z
readout, <Z> = cos(theta); with theta = arccos(a) this is a, with theta = arcsin(a) + pi/2 it is -a.
Only the closed forms are evaluated here (no simulator is called)."""
import json
import os

a = [-1.0, -0.75, -0.3, 0.0, 0.2, 0.5, 0.9, 1.0]
out = {
    "_source": "caption of the input-scaling figure, section 'QPINN architecture and ansatz designs'",
    "a": a,
    "acos_expect_z": a,
    "asin_expect_z": [-v for v in a],
}
with open(os.path.join(os.path.dirname(__file__), "scaling_identities.json"), "w") as fh:
    json.dump(out, fh, indent=1)
