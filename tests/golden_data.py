"""Readers of the stored expected values under tests/golden/ (text fixtures; each file states its source)."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def philox_kat():
    """[(counter[4], key[2], output[4])] from the published Philox4x32-10 known-answer list."""
    out = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(t, 16) for t in line.split()]
            assert len(w) == 10
            out.append((w[0:4], w[4:6], w[6:10]))
    return out


def fa_landau(name="fa_landau_12x6x4x8_seed11.txt"):
    """An FA fixture: dict with dims, seed, alpha, eps, input_plaquette, input_F, history [(k, theta, F)],
    tol, iters_to_tol, final_theta, final_F (and final_plaquette where the file has it)."""
    from paper_1208_1186_amd import synth
    d = {"history": [], "eps": synth.EPS_P059}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            if line.startswith("# input:"):
                cfg = line.split("make_config(")[1].split(")")
                d["dims"] = tuple(int(v) for v in cfg[0].strip("(").split(","))
                d["seed"] = int(cfg[1].strip(", "))
                d["alpha"] = float(line.split("alpha =")[1])
                continue
            if line.startswith("# eps "):
                d["eps"] = float(line.split("=")[1])
                continue
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            if t[0].isdigit():
                d["history"].append((int(t[0]), float(t[1]), float(t[2])))
            elif t[0] == "iters_to_tol":
                d[t[0]] = int(t[1])
            else:
                d[t[0]] = float(t[1])
    return d
