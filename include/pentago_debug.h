/*
 * pentago_debug.h -- host-side self-check entry points of the library.
 *
 * These run the library's own rotation-abstracted primitives (the same
 * source the GPU kernels are compiled from) on the host CPU, so that they can
 * be checked against their definitions without a GPU.  Sets use the layout
 * of pentago_set256 (bit g of L in word g >> 6 at position g & 63).
 */
#ifndef PENTAGO_DEBUG_H
#define PENTAGO_DEBUG_H

#include <stdint.h>

#include "pentago.h"

#ifdef __cplusplus
extern "C" {
#endif

/* The set of g in L for which g.board has five in a row of colour (1 black,
 * 2 white) (Section III). */
int pentago_debug_five(pentago_board board, int color, pentago_set256 *out);

/* rmax(in)(g) = OR over the 8 single-quadrant turns r of in(g + r) (Section III). */
int pentago_debug_rmax(const pentago_set256 *in, pentago_set256 *out);

/* out(g) = in(g - k e_d): the table of a board whose quadrant d is turned k
 * more times counter-clockwise (Section III, f_b -> f_gb for g in L). */
int pentago_debug_shift(const pentago_set256 *in, int d, int k, pentago_set256 *out);

/* out(g') = in(g) where g' is g with coordinates d and 3 exchanged: the
 * internal layout the sweep kernels work in when quadrant d receives the
 * stones (self-inverse; identity for d = 3). */
int pentago_debug_swap3(const pentago_set256 *in, int d, pentago_set256 *out);

/* The image of a table under board symmetry sym (numbered as in
 * pentago_section_image): out(G) = in(g) with g_i = sign * (G_{pi(i)} - h[pi(i)]),
 * where pi moves quadrant i to quadrant pi(i), sign is -1 for the reflections
 * (sym >= 4) and h[j] are the turns of image quadrant j (Section III). */
int pentago_debug_sym(const pentago_set256 *in, int sym, const int h[4], pentago_set256 *out);

/* The pattern map of board symmetry sym for the (black, white) class: image
 * pattern `index` comes from source pattern *src_index, whose local image
 * (mirror if sym >= 4, then sym & 3 counter-clockwise turns) is the image
 * pattern turned *h more times (Section III). */
int pentago_debug_sym_pattern(int sym, int black, int white, int index, int *src_index, int *h);

/* Rotation-minimal pattern of a quadrant code: its index in its (black,
 * white) class and the least number of counter-clockwise turns k taking the
 * code to it (Section IV). */
int pentago_debug_canon(int code, int *index, int *k);

#ifdef __cplusplus
}
#endif

#endif
