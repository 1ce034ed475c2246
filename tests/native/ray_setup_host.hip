// Host driver for the library's ray set-up (fpo_device.h: setup_ray_in,
// setup_ray, tree_dev), which is host-callable.  Reads one ray and box per
// line from stdin: ox oy oz dx dy dz lo_x lo_y lo_z hi_x hi_y hi_z (FP32
// values written exactly); writes per line: hit t_in t_len entry_x entry_y
// entry_z same_as_cube, where same_as_cube is 1 if the box is the unit cube
// and the result equals setup_ray's bit for bit (0 if it differs, - if the
// box is another one).  First line of output: the box tree_dev derives from
// lattice bounds (161, 174, 176, 347, 349, 332) at depth 9, and from none.
#include <cstdio>
#include <cstring>

#include "fpo_device.h"

using fpo::dev::Ray;

int main()
{
    fpo_tree_view v;
    std::memset(&v, 0, sizeof(v));
    v.max_depth = 9;
    const int32_t b[6] = {161, 174, 176, 347, 349, 332};
    v.bounds = b;
    const fpo::dev::TreeDev a = fpo::dev::tree_dev(&v);
    v.bounds = nullptr;
    const fpo::dev::TreeDev c = fpo::dev::tree_dev(&v);
    std::printf("tree_dev %.9g %.9g %.9g %.9g %.9g %.9g | %.9g %.9g %.9g %.9g %.9g %.9g\n", a.box_lo[0], a.box_lo[1],
                a.box_lo[2], a.box_hi[0], a.box_hi[1], a.box_hi[2], c.box_lo[0], c.box_lo[1], c.box_lo[2], c.box_hi[0],
                c.box_hi[1], c.box_hi[2]);
    float x[12];
    while (std::scanf("%g %g %g %g %g %g %g %g %g %g %g %g", &x[0], &x[1], &x[2], &x[3], &x[4], &x[5], &x[6], &x[7],
                      &x[8], &x[9], &x[10], &x[11]) == 12) {
        Ray r;
        std::memset(&r, 0, sizeof(r));
        const bool hit = fpo::dev::setup_ray_in(x + 6, x + 9, x[0], x[1], x[2], x[3], x[4], x[5], r);
        const bool cube = x[6] == 0.0f && x[7] == 0.0f && x[8] == 0.0f && x[9] == 1.0f && x[10] == 1.0f && x[11] == 1.0f;
        const char* same = "-";
        if (cube) {
            Ray q;
            std::memset(&q, 0, sizeof(q));
            const bool hq = fpo::dev::setup_ray(x[0], x[1], x[2], x[3], x[4], x[5], q);
            same = (hq == hit && std::memcmp(&q, &r, sizeof(Ray)) == 0) ? "1" : "0";
        }
        std::printf("%d %.9g %.9g %.9g %.9g %.9g %s\n", hit ? 1 : 0, r.t_in, r.t_len, r.o[0], r.o[1], r.o[2], same);
    }
    return 0;
}
