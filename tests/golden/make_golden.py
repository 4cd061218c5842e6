"""Write the stored expected values under tests/golden/ (run by hand).

Every value here comes from the seeded generators in ``synth`` and the CPU
oracle in ``oracle``; nothing is read from the GPU library.

  python tests/golden/make_golden.py
"""

import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402
from oracle import workload  # noqa: E402


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def synth_hashes():
    wl = synth.tiny_workload()
    out = {
        "vessel_pos": sha(wl.mesh.pos), "vessel_nrm": sha(wl.mesh.nrm),
        "vessel_uv": sha(wl.mesh.uv), "vessel_tri": sha(wl.mesh.tri),
        "tiny_cameras": sha(np.stack(wl.cameras)),
        "tiny_brush_centres": sha(np.stack([e.centre for e in wl.edits if e.kind == "brush"])),
        "tiny_polys": sha(np.concatenate([e.poly for e in wl.edits if e.kind == "lasso"])),
        "tiny_kinds": "".join("b" if e.kind == "brush" else "l" for e in wl.edits),
    }
    return out


def tiny_oracle():
    wl = synth.tiny_workload()
    geom, layers, areas = workload.run(wl)
    return {
        "workload": "vessel 128^2 vertices (32,258 tris), 512^2 atlas, 64 edits",
        "covered_texels": int((geom.tri_id >= 0).sum()),
        "total_area": float(geom.w.sum()),
        "layer_sha256": sha(layers[0]),
        "label_counts": np.bincount(layers[0], minlength=8)[:8].tolist(),
        "areas": [float(a) for a in areas[0][:8]],
    }


if __name__ == "__main__":
    oracle.build(force=False)
    with open(os.path.join(HERE, "synth_sha256.json"), "w") as f:
        json.dump(synth_hashes(), f, indent=1)
    with open(os.path.join(HERE, "vessel512_oracle.json"), "w") as f:
        json.dump(tiny_oracle(), f, indent=1)
    print("written")
