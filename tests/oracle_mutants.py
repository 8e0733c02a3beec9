"""Mutation check of the oracle's pins (CPU only; not collected by pytest).

Each mutant plants one plausible mistake in a copy of oracle/gd_oracle.c (a dropped term,
a wrong sign, index or comparison, a missing rule), builds it, and runs the oracle's pin
tests (tests/test_oracle_*.py) against it.  A mutant that no pin kills is reported as a
survivor: a part of the oracle that nothing outside the oracle itself checks.

    python tests/oracle_mutants.py [--workdir DIR] [--jobs N] [--only NAME ...]

Exit status 0 when every mutant is killed.
"""
from __future__ import annotations

import argparse
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "gd_oracle.c")

# (name, exact text in the source, replacement); each text occurs exactly once
MUTANTS = [
    # dynamics (App. B)
    ("bicycle full-step speed for the position", "double vbar = clipd(*v + 0.5 * a * dt, -vmax, vmax);",
     "double vbar = clipd(*v + a * dt, -vmax, vmax);"),
    ("bicycle slip angle without l_r = L/2", "double beta = atan(0.5 * tan(steer));",
     "double beta = atan(tan(steer));"),
    ("bicycle yaw rate without cos(beta)", "double thd = vbar * cos(beta) * tan(steer) / L;",
     "double thd = vbar * tan(steer) / L;"),
    ("bicycle speed not clipped", "double vn = clipd(*v + a * dt, -vmax, vmax);", "double vn = *v + a * dt;"),
    ("bicycle heading without slip", "double xd = vbar * cos(*yaw + beta);", "double xd = vbar * cos(*yaw);"),
    ("simplified model without the acceleration term", "double d = *v * dt + 0.5 * a * dt * dt;\n    double th = *yaw;",
     "double d = *v * dt;\n    double th = *yaw;"),
    ("simplified model yaw from the start speed", "*yaw = th + s * d;", "*yaw = th + s * *v * dt;"),
    # collision
    ("box/box SAT with one box's axes only", "for (int k = 0; k < 2; k++) {\n        double c = cos(boxes[k][2])",
     "for (int k = 0; k < 1; k++) {\n        double c = cos(boxes[k][2])"),
    ("box/segment SAT without the segment normal", "        naxes = 3;\n", "        naxes = 2;\n"),
    ("parked agents not collided with", "if (j == i || !(b->flags[j] & (OR_ALIVE | OR_STATIC))) continue;",
     "if (j == i || !(b->flags[j] & OR_ALIVE)) continue;"),
    ("pedestrians collide with edges", "        if (b->cls && b->cls[i] == OR_CLASS_PEDESTRIAN) continue;\n", ""),
    ("edge segments across polylines", "return (meta[k] & 0xff) == OR_TYPE_EDGE && !(meta[k] & OR_META_LAST);",
     "return (meta[k] & 0xff) == OR_TYPE_EDGE;"),
    ("touching boxes collide", "if (sep < 0.0) coll[i - a0] |= OR_COLL_AGENT;", "if (sep <= 1e-3) coll[i - a0] |= OR_COLL_AGENT;"),
    # reward, done, reset
    ("collision penalty added", "r = (goal ? 1.0 : 0.0) - (collided ? c->collision_penalty : 0.0);",
     "r = (goal ? 1.0 : 0.0) + (collided ? c->collision_penalty : 0.0);"),
    ("no termination on collision", "done = goal || ((c->flags & OR_TERM_ON_COLLISION) && collided) || last;",
     "done = goal || last;"),
    ("episode one step too long", "int last = b->t[w] + 1 >= c->episode_len;", "int last = b->t[w] + 1 > c->episode_len;"),
    ("world not done when every agent is", "int wdone = !any_alive || last;", "int wdone = last;"),
    ("reset drops the step's outcome", "uint8_t keep = b->flags[i] & (OR_COLL_AGENT | OR_COLL_EDGE | OR_GOAL | OR_DONE);",
     "uint8_t keep = 0;"),
    ("parked agents finish", "            out = OR_VISIBLE | OR_STATIC;\n            done = 0;",
     "            out = OR_VISIBLE | OR_STATIC;\n            done = 1;"),
    ("no parking", "            return OR_VISIBLE | OR_STATIC;", "            return OR_ALIVE | OR_VISIBLE;"),
    # observation decisions
    ("strict radius (FP64)", "return key64(px, py, qx, qy) <= r * r;", "return key64(px, py, qx, qy) < r * r;"),
    ("strict radius (binary32)", "<= r2_32(r);", "< r2_32(r);"),
    ("road ties to the highest index", "return (a->idx > b->idx) - (a->idx < b->idx);",
     "return (a->idx < b->idx) - (a->idx > b->idx);"),
    ("ego collision entries at episode start", "ego[5] = (!fresh && (b->flags[i] & OR_COLL_AGENT)) ? 1.0 : 0.0;",
     "ego[5] = (b->flags[i] & OR_COLL_AGENT) ? 1.0 : 0.0;"),
    ("ego goal y' sign", "ego[4] = -st * gdx + ct * gdy;", "ego[4] = st * gdx + ct * gdy;"),
    ("partner slot order", "int j = a0 + (s < l ? s : s + 1);", "int j = a0 + (s <= l ? s : s + 1);"),
    ("partner heading reversed", "f[2] = wrap_angle(b->yaw[j] - th);", "f[2] = wrap_angle(th - b->yaw[j]);"),
    ("removed agents observed as partners", "            if (!(b->flags[j] & OR_VISIBLE)) continue;\n            double d64", "            double d64"),
    ("road direction not in the ego frame", "road[q * 4 + 2] = wrap_angle(b->rdir[k] - th);", "road[q * 4 + 2] = wrap_angle(b->rdir[k]);"),
    # LIDAR
    ("ring not turned with the heading", ": th + 2.0 * OR_PI * (double)k / (double)N;", ": 2.0 * OR_PI * (double)k / (double)N;"),
    ("own box seen by the LIDAR", "if (j == i || !(b->flags[j] & OR_VISIBLE)) continue;\n                double cr[4][2];",
     "if (!(b->flags[j] & OR_VISIBLE)) continue;\n                double cr[4][2];"),
    ("cone rays at sub-arc edges", "c->lidar_fov * (((double)k + 0.5) / (double)N - 0.5)", "c->lidar_fov * ((double)k / (double)N - 0.5)"),
    # smooth reward and its VJP
    ("nearest edge beyond the radius", "if (bestk >= 0 && best <= c->obs_radius) {", "if (bestk >= 0) {"),
    ("nearest edge ties to the highest index", "        if (d < best) {\n            best = d;\n            bestk = k;",
     "        if (d <= best) {\n            best = d;\n            bestk = k;"),
    ("off-road side reversed", "return cr < 0.0 ? 1.0 : -1.0;", "return cr > 0.0 ? 1.0 : -1.0;"),
    ("softplus without its smooth part", "(z > 0.0 ? z : 0.0) + log1p(exp(-fabs(z)))", "(z > 0.0 ? z : 0.0)"),
    ("goal distance along one axis", "    double ng = sqrt(gpx * gpx + gpy * gpy);\n    double s;",
     "    double ng = sqrt(gpx * gpx);\n    double s;"),
    ("VJP slip derivative without its denominator", "double dbeta = 0.5 * sec2 / (1.0 + 0.25 * tdl * tdl);",
     "double dbeta = 0.5 * sec2;"),
    ("VJP acceleration through the midpoint speed", "double ba = bvb * c1 * 0.5 * dt + lv * c2 * dt;",
     "double ba = bvb * c1 * dt + lv * c2 * dt;"),
    ("VJP simplified-model curvature", "grad_actions[((int64_t)t * A + i) * 2 + 1] = lth * d;",
     "grad_actions[((int64_t)t * A + i) * 2 + 1] = lth;"),
    ("VJP goal term sign", "lx += -ct * bgx + st * bgy;", "lx += ct * bgx + st * bgy;"),
    # rollout observation and its VJP
    ("rollout obs goal in the world frame", "                o[1] = ct * dxg + st * dyg;", "                o[1] = dxg;"),
    ("rollout obs partner radius exclusive", "                    if (dx * dx + dy * dy > R * R) continue;",
     "                    if (dx * dx + dy * dy >= R * R) continue;"),
    ("rollout obs heading difference reversed", "const double dyaw = wrap_angle(S[2 * A + jj] - th);",
     "const double dyaw = wrap_angle(th - S[2 * A + jj]);"),
    ("obs VJP without the partner's position term", "                        Dj[0] += rx;\n                        Dj[1] += ry;\n", ""),
    ("obs VJP rotation term sign", "Di[2] += bx * fy - by * fx;", "Di[2] -= bx * fy - by * fx;"),
    ("obs VJP without the partner's speed", "                        Dj[3] += bv;\n", ""),
    # inversion and decimation
    ("inversion of a standing vehicle", "double st = fabs(d) < OR_INV_MIN_DIST ? 0.0 : w / d;", "double st = w / d;"),
    ("inversion without the heading wrap", "double w = wrap_angle(dth);", "double w = dth;"),
    ("decimation ties to the highest index", "if (best < 0 || a < ba) {", "if (best < 0 || a <= ba) {"),
    ("decimation removes points at the threshold", "if (best < 0 || !(ba < min_area)) break;",
     "if (best < 0 || !(ba <= min_area)) break;"),
]


def run_one(name, old, new, workdir, idx):
    src = open(SRC).read()
    if src.count(old) != 1:
        return name, "not applicable (text occurs %d times)" % src.count(old)
    d = os.path.join(workdir, "m%02d" % idx)
    os.makedirs(d, exist_ok=True)
    msrc = os.path.join(d, "gd_oracle.c")
    with open(msrc, "w") as f:
        f.write(src.replace(old, new))
    lib = os.path.join(d, "liboracle.so")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-w",
                           "-o", lib, msrc, "-lm"])
    env = dict(os.environ, GD_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    tests = sorted(os.path.join(ROOT, "tests", t) for t in os.listdir(os.path.join(ROOT, "tests"))
                   if t.startswith("test_oracle_"))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *tests],
                       cwd=ROOT, env=env, capture_output=True, text=True)
    if r.returncode == 0:
        return name, "SURVIVED"
    failed = [ln.split(" ")[1] for ln in r.stdout.splitlines() if ln.startswith("FAILED")]
    return name, "killed by " + (failed[0] if failed else "an error (rc %d)" % r.returncode)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workdir", default=None)
    ap.add_argument("--jobs", type=int, default=4)
    ap.add_argument("--only", nargs="*", default=None)
    args = ap.parse_args()
    tmp = None
    if args.workdir is None:
        tmp = tempfile.TemporaryDirectory()
        args.workdir = tmp.name
    todo = [(i, m) for i, m in enumerate(MUTANTS) if not args.only or any(o in m[0] for o in args.only)]
    with ThreadPoolExecutor(args.jobs) as ex:
        res = list(ex.map(lambda im: run_one(*im[1], args.workdir, im[0]), todo))
    survivors = 0
    for name, verdict in res:
        print("%-50s %s" % (name, verdict))
        survivors += verdict == "SURVIVED" or verdict.startswith("not applicable")
    print("%d mutants, %d survived or not applicable" % (len(res), survivors))
    return 1 if survivors else 0


if __name__ == "__main__":
    sys.exit(main())
