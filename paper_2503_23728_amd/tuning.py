"""On-disk cache of autotuned launch shapes.

pimd_autotune times the candidate launch shapes of the force kernels on the
live state; the winner depends on the GPU and on the batch (atoms, beads and
box of every ring polymer, the descriptor and network sizes, the precision).
The cache maps a key of exactly those inputs to the chosen shape, so the sweep
runs once per machine and workload and later contexts reapply its result.

Location: $PIMD_TUNING_CACHE, else ~/.cache/paper_2503_23728_amd/tuning.json.
"""
import hashlib
import json
import os

FIELDS = ("centre_waves", "centre_grid", "mlp_rows", "neighbor_cells", "mlp_waves", "force_rows", "centre_lanes",
          "mlp_chain")


def cache_path():
    p = os.environ.get("PIMD_TUNING_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2503_23728_amd", "tuning.json")


def config_key(arch, n_cu, systems, model, precision, max_neighbors, neighbor_skin=0.0):
    """Hash of everything the fastest launch shape can depend on."""
    desc = {
        "arch": arch, "cu": int(n_cu), "precision": precision, "kmax": int(max_neighbors),
        "systems": sorted([int(s.n_atoms), int(s.n_beads), [round(float(b), 4) for b in s.box]] for s in systems),
    }
    if model is not None and hasattr(model, "width"):      # direct-force head
        desc["model"] = {"head": "gfn", "elements": int(model.n_elements), "n_rad": int(model.n_rad),
                         "width": int(model.width), "layers": int(model.n_layers), "cutoff": float(model.cutoff)}
    elif model is not None:
        desc["model"] = {"elements": int(model.n_elements), "n_rad": int(model.n_rad),
                         "n_ang_eta": len(model.ang_eta), "hidden": [int(h) for h in model.hidden],
                         "cutoff": float(model.cutoff)}
        if getattr(model, "angular", "g4") != "g4":
            desc["model"]["angular"] = model.angular
    if neighbor_skin:
        desc["skin"] = round(float(neighbor_skin), 4)
    blob = json.dumps(desc, sort_keys=True).encode()
    return hashlib.sha256(blob).hexdigest()[:32]


def _read(path):
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def load(key, path=None):
    """The cached shape for key ({field: int}) or None."""
    entry = _read(path or cache_path()).get(key)
    if not isinstance(entry, dict) or not all(isinstance(entry.get(f), int) for f in FIELDS):
        return None
    return {f: entry[f] for f in FIELDS}


def store(key, shape, path=None, extra=None):
    """Record shape under key; returns False when the cache cannot be written."""
    path = path or cache_path()
    data = _read(path)
    data[key] = dict({f: int(shape[f]) for f in FIELDS}, **(extra or {}))
    try:
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        tmp = f"{path}.{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
        return True
    except OSError:
        return False
