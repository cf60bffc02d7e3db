"""Write the workload models (chain3, quadruped, humanoid, arm_box and the joint-limited
chain3_lim, quadruped_lim, humanoid_lim, the quadruped and humanoid on random-height grids of box tiles, the damped chain3_damp and
humanoid_damp, quadruped_slip with frictionless feet, and quadruped_hfield on height-field terrain)
as JSON files in the form rb_model_create_json reads.  The generators in workloads/robots.py are the source; the
files are for callers that load a model without Python."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from workloads import robots  # noqa: E402

NAMES = ("chain3", "quadruped", "humanoid", "arm_box", "chain3_lim", "quadruped_lim", "humanoid_lim",
         "quadruped_terrain", "humanoid_terrain", "chain3_damp", "humanoid_damp", "quadruped_slip", "quadruped_hfield",
         "chain3_loop", "humanoid_weld", "quadruped_condim6", "humanoid_condim4",
         "quadruped_elliptic", "humanoid_elliptic", "cube_stack", "pincer", "humanoid_self", "pincer_cube",
         "quadruped_elliptic4", "humanoid_elliptic4", "quadruped_elliptic6")


def main():
    for name in NAMES:
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(robots.by_name(name), f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main()
