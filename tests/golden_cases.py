"""Parser for tests/golden/hand_cases.txt (hand-derived expected outputs)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hand_cases.txt")


def load_cases(path=GOLDEN):
    cases = []
    cur = None
    with open(path) as f:
        for raw in f:
            line = raw.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split(None, 1)
            if tok[0] == "case":
                cur = dict(name=tok[1], hits=[], expect=[])
            elif tok[0] == "cite":
                cur["cite"] = tok[1]
            elif tok[0] == "params":
                v = [float(s) for s in tok[1].split()]
                cur["params"] = dict(dc=v[0], rho_c=v[1], delta_c=v[2], delta_o=v[3],
                                     bounds=(v[4], v[5], v[6], v[7]), n_layers=int(v[8]))
            elif tok[0] == "hit":
                lhs, rhs = tok[1].split("|")
                a = lhs.split()
                b = rhs.split()
                cur["hits"].append((float(a[0]), float(a[1]), int(a[2]), float(a[3])))
                cur["expect"].append((float(b[0]), int(b[1]), int(b[2]), int(b[3])))
            elif tok[0] == "followers":
                # F_i of Eq. 5 for one owner i, or "none": every list empty
                cur.setdefault("followers", {})
                if tok[1].strip() != "none":
                    owner, rest = tok[1].split(":")
                    cur["followers"][int(owner)] = [int(v) for v in rest.split()]
            elif tok[0] == "end":
                h = cur["hits"]
                e = cur["expect"]
                cur["event"] = dict(
                    x=np.array([t[0] for t in h], np.float32),
                    y=np.array([t[1] for t in h], np.float32),
                    layer=np.array([t[2] for t in h], np.int32),
                    energy=np.array([np.float32(t[3]) for t in h], np.float32),
                )
                cur["rho"] = np.array([np.float32(t[0]) for t in e], np.float32)
                cur["nh"] = np.array([t[1] for t in e], np.int32)
                cur["cluster_id"] = np.array([t[2] for t in e], np.int32)
                cur["is_seed"] = np.array([t[3] for t in e], np.uint8)
                assert "followers" in cur, f"case {cur['name']} states no follower lists"
                fs = [0]
                fl = []
                for i in range(len(h)):
                    fl.extend(cur["followers"].get(i, []))
                    fs.append(len(fl))
                cur["fstart"] = np.array(fs, np.int32)
                cur["flist"] = np.array(fl, np.int32)
                cases.append(cur)
                cur = None
    return cases
